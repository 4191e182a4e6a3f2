// Host mesh builder (FP64): orientation, face connectivity, geometric factors, normals,
// face-node maps, locality order and the packed per-element records used by the kernels.
//
// Sec. 2: each element is the affine image of the reference tetrahedron, so the global
// operators are the reference ones scaled by per-element constants (eq.
// dg-reference-matrices). Sec. 5.3: the flux gather reads the facial nodes of the element
// and of its neighbour through small index lists, and the element numbering is chosen for
// the locality of that gather.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "refops.hpp"

namespace dgh {

// Per-element geometric record, in this order (kGeoStride values):
//   0..8   rx ry rz sx sy sz tx ty tz   (d r_mu / d x_nu, constant per element)
//   9..24  per face f: nx ny nz Fscale  (outward unit normal and sJ/J)
//   25     J
constexpr int kGeoStride = 26;
constexpr int kGeoNormal = 9;
constexpr int kGeoJ = 25;

// Packed face record: kFacePec for a perfectly conducting wall, kFaceAbsorbing for an
// absorbing face (zero exterior state), kFaceScatter0 - i for scatterer face i (a wall for the
// total field of the scattered-field form: E+ = -E- - 2 E_inc, H+ = H-), else
// (neighbour internal id << 5) | (orientation code << 2) | neighbour face.
constexpr int32_t kFacePec = -1;
constexpr int32_t kFaceAbsorbing = -2;
constexpr int32_t kFaceScatter0 = -3;
inline int32_t pack_face(int32_t nbr, int orient, int nface) {
  return (nbr << 5) | (orient << 2) | nface;
}

// Per-element material record of a heterogeneous medium (kMatStride values):
//   0 1/eps  1 1/mu  2 eps  3 mu
//   4..19  per face f: A B C D, the impedance-weighted upwind flux of Sec. 6 folded with
//          Fscale and the inverse material constants:
//            Fscale/eps [n.F - (n.F)*]_E = A n x [H] + B ([E] - (n.[E]) n)
//            Fscale/mu  [n.F - (n.F)*]_H = -C n x [E] + D ([H] - (n.[H]) n)
//          A = Fscale/eps Z+/(Z- + Z+), B = Fscale/eps 1/(Z- + Z+),
//          C = Fscale/mu  Y+/(Y- + Y+), D = Fscale/mu  1/(Y- + Y+),  Z = sqrt(mu/eps), Y = 1/Z,
//          and Z+ = Z- on walls and absorbing faces.
constexpr int kMatStride = 20;
constexpr int kMatFace = 4;

struct MeshData {
  int K = 0;
  std::vector<int32_t> etov;         // K x 4 after the orientation fix (user order)
  std::vector<int32_t> etoe, etof;   // K x 4 (user order); boundary faces point to themselves
  std::vector<int32_t> orient;       // K x 4 orientation code of interior faces, -1 on walls
  std::vector<int8_t> wall_kind;     // K x 4 (user order, internal face numbering): face_bc
                                     // of a boundary face (0 automatic, 1 wall, 2 absorbing,
                                     // 3 scatterer), 0 on interior faces
  std::vector<int32_t> scat_face;    // scatterer faces in face-record order: internal
                                     // element * 4 + face
  std::vector<double> geo;           // K x kGeoStride (user order)
  std::vector<double> x;             // 3 x K x Np physical node coordinates (user order)
  std::vector<int32_t> elem_of;      // internal position -> user element
  std::vector<int32_t> pos_of;       // user element -> internal position
  std::vector<int32_t> face_code;    // K x 4 packed face records in internal order
};

// Throws std::runtime_error with a message on an invalid mesh (degenerate element, a face
// shared by more than two elements, bad vertex id). face_bc (K x 4 or null) is indexed by the
// faces of etov as given: 0 automatic (wall if unmatched), 1 wall, 2 absorbing, 3 scatterer
// (a wall for the total field of the scattered-field form). group (K or
// null): elements of one group stay contiguous, in group order, under the locality order.
MeshData build_mesh(const RefOps& R, int nverts, const double* vxyz, int K, const int32_t* etov,
                    const int8_t* face_bc, int reorder, const int32_t* group = nullptr);

// Material records (K x kMatStride, internal order) for per-element eps, mu (user order; a
// null array means 1). Throws on a value that is not finite and positive.
std::vector<double> material_records(const MeshData& m, const double* eps, const double* mu);

// Canonical face maps (user order, reference node order): flat node ids k*Np + n.
void canonical_maps(const RefOps& R, const MeshData& m, int32_t* vmapM, int32_t* vmapP);

}  // namespace dgh

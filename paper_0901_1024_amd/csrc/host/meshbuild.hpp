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

// Packed face record: -1 for a perfectly conducting wall, else
// (neighbour internal id << 5) | (orientation code << 2) | neighbour face.
inline int32_t pack_face(int32_t nbr, int orient, int nface) {
  return (nbr << 5) | (orient << 2) | nface;
}

struct MeshData {
  int K = 0;
  std::vector<int32_t> etov;         // K x 4 after the orientation fix (user order)
  std::vector<int32_t> etoe, etof;   // K x 4 (user order); boundary faces point to themselves
  std::vector<int32_t> orient;       // K x 4 orientation code of interior faces, -1 on walls
  std::vector<double> geo;           // K x kGeoStride (user order)
  std::vector<double> x;             // 3 x K x Np physical node coordinates (user order)
  std::vector<int32_t> elem_of;      // internal position -> user element
  std::vector<int32_t> pos_of;       // user element -> internal position
  std::vector<int32_t> face_code;    // K x 4 packed face records in internal order
};

// Throws std::runtime_error with a message on an invalid mesh (degenerate element, a face
// shared by more than two elements, bad vertex id).
MeshData build_mesh(const RefOps& R, int nverts, const double* vxyz, int K, const int32_t* etov,
                    const int8_t* face_bc, int reorder);

// Canonical face maps (user order, reference node order): flat node ids k*Np + n.
void canonical_maps(const RefOps& R, const MeshData& m, int32_t* vmapM, int32_t* vmapP);

}  // namespace dgh

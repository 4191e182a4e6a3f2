// Reference-element operators for nodal DG on tetrahedra, built on the host in FP64.
//
// Sec. 2 of the paper: Lagrange basis on interpolation nodes, reference mass,
// differentiation and face-mass matrices (eqs. dg-global-matrices, dg-reference-matrices)
// and the lifting matrix L = M^-1 [M^A1 .. M^A4] (Fig. lifting-matrix).
#pragma once

#include <array>
#include <vector>

namespace dgh {

// Local vertex triples of the reference faces F1..F4 and the opposite vertex of each.
// F1 = (v1,v2,v3) t=-1, F2 = (v1,v2,v4) s=-1, F3 = (v2,v3,v4) r+s+t=-1, F4 = (v1,v3,v4) r=-1.
constexpr int kFaceVerts[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {0, 2, 3}};
constexpr int kFaceOpposite[4] = {3, 2, 0, 1};
// The six orderings of three face vertices; a face-pair orientation code indexes this list.
constexpr int kPerm3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

struct RefOps {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> r, s, t;              // nodes, Np each
  std::vector<std::array<int, 4>> bary;     // integer barycentrics (N-i-j-k, i, j, k)
  std::vector<double> Dr, Ds, Dt;           // Np x Np, row-major
  std::vector<double> M;                    // mass, Np x Np
  std::vector<double> LIFT;                 // Np x 4Nfp, row-major
  std::vector<int> Fmask;                   // 4 x Nfp, ascending node ids per face
  // Face-node correspondence across an interior face: for my face f, the neighbour's face
  // f2, orientation code o (kPerm3 index mapping my face vertex a to the neighbour's face
  // vertex kPerm3[o][a]) and my face node j, the neighbour's volume node id.
  std::vector<int> nbr_node;                // [4][4][6][Nfp]
};

// Throws std::runtime_error on an unsupported order or a singular matrix.
RefOps build_ref_ops(int N);

// Dense helpers (row-major, n x n).
bool invert(std::vector<double>& a, int n);

}  // namespace dgh

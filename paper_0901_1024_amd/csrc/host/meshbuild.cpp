// Host mesh builder (FP64). See meshbuild.hpp.
#include "meshbuild.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>
#include <stdexcept>

namespace dgh {
namespace {

// Spread the low 21 bits of v so that two zero bits follow each bit (3D Morton interleave).
uint64_t spread3(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | (v << 32)) & 0x1f00000000ffffULL;
  v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
  v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
  v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
  v = (v | (v << 2)) & 0x1249249249249249ULL;
  return v;
}

}  // namespace

MeshData build_mesh(const RefOps& R, int nverts, const double* vxyz, int K, const int32_t* etov_in,
                    const int8_t* face_bc, int reorder, const int32_t* group) {
  if (K <= 0 || nverts < 4) throw std::runtime_error("empty mesh");
  if (K >= (1 << 26)) throw std::runtime_error("too many elements for the packed face record");
  MeshData m;
  m.K = K;
  m.etov.assign(etov_in, etov_in + size_t(K) * 4);
  for (int64_t q = 0; q < int64_t(K) * 4; ++q)
    if (m.etov[q] < 0 || m.etov[q] >= nverts) throw std::runtime_error("vertex id out of range");

  // Orientation: det[v2-v1, v3-v1, v4-v1] must be positive; a negative one swaps v3 and v4
  // (which exchanges the faces F1 = (v1,v2,v3) and F2 = (v1,v2,v4)).
  std::vector<uint8_t> swapped(K, 0);
  for (int k = 0; k < K; ++k) {
    const double* p[4];
    for (int v = 0; v < 4; ++v) p[v] = vxyz + 3 * size_t(m.etov[size_t(k) * 4 + v]);
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) a[d] = p[1][d] - p[0][d], b[d] = p[2][d] - p[0][d], c[d] = p[3][d] - p[0][d];
    double det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                 a[2] * (b[0] * c[1] - b[1] * c[0]);
    if (det == 0.0 || !std::isfinite(det)) throw std::runtime_error("degenerate element");
    if (det < 0.0) {
      std::swap(m.etov[size_t(k) * 4 + 2], m.etov[size_t(k) * 4 + 3]);
      swapped[k] = 1;
    }
  }

  // Connectivity: sort faces by their sorted vertex triple; equal neighbours pair up.
  struct FaceKey {
    int32_t a, b, c;
    int32_t slot;  // k*4 + f
  };
  std::vector<FaceKey> keys(size_t(K) * 4);
  for (int k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      int32_t v[3];
      for (int q = 0; q < 3; ++q) v[q] = m.etov[size_t(k) * 4 + kFaceVerts[f][q]];
      std::sort(v, v + 3);
      keys[size_t(k) * 4 + f] = {v[0], v[1], v[2], k * 4 + f};
    }
  std::sort(keys.begin(), keys.end(), [](const FaceKey& x, const FaceKey& y) {
    if (x.a != y.a) return x.a < y.a;
    if (x.b != y.b) return x.b < y.b;
    if (x.c != y.c) return x.c < y.c;
    return x.slot < y.slot;
  });
  m.etoe.resize(size_t(K) * 4);
  m.etof.resize(size_t(K) * 4);
  for (int k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) m.etoe[size_t(k) * 4 + f] = k, m.etof[size_t(k) * 4 + f] = f;
  auto same = [](const FaceKey& x, const FaceKey& y) { return x.a == y.a && x.b == y.b && x.c == y.c; };
  for (size_t q = 0; q < keys.size();) {
    size_t e = q + 1;
    while (e < keys.size() && same(keys[q], keys[e])) ++e;
    if (e - q > 2) throw std::runtime_error("non-conforming mesh: a face is shared by more than two elements");
    if (e - q == 2) {
      int s1 = keys[q].slot, s2 = keys[q + 1].slot;
      m.etoe[s1] = s2 / 4, m.etof[s1] = s2 % 4;
      m.etoe[s2] = s1 / 4, m.etof[s2] = s1 % 4;
    }
    q = e;
  }
  m.wall_kind.assign(size_t(K) * 4, 0);
  if (face_bc) {
    for (int k = 0; k < K; ++k)
      for (int fu = 0; fu < 4; ++fu) {
        const int8_t bc = face_bc[size_t(k) * 4 + fu];
        const int f = swapped[k] && fu < 2 ? 1 - fu : fu;   // the user's face in internal numbering
        const size_t q = size_t(k) * 4 + f;
        const bool boundary = m.etoe[q] == k && m.etof[q] == f;
        if (bc < 0 || bc > 3) throw std::runtime_error("unsupported face condition");
        if (bc != 0 && !boundary) throw std::runtime_error("boundary condition on an interior face");
        m.wall_kind[q] = bc;
      }
  }

  // Orientation code of each interior face: my face vertex a is the neighbour's face vertex
  // kPerm3[o][a].
  m.orient.assign(size_t(K) * 4, -1);
  for (int k = 0; k < K; ++k)
    for (int f = 0; f < 4; ++f) {
      size_t q = size_t(k) * 4 + f;
      int k2 = m.etoe[q], f2 = m.etof[q];
      if (k2 == k && f2 == f) continue;
      int mine[3], theirs[3];
      for (int a = 0; a < 3; ++a) {
        mine[a] = m.etov[size_t(k) * 4 + kFaceVerts[f][a]];
        theirs[a] = m.etov[size_t(k2) * 4 + kFaceVerts[f2][a]];
      }
      int code = -1;
      for (int o = 0; o < 6 && code < 0; ++o)
        if (mine[0] == theirs[kPerm3[o][0]] && mine[1] == theirs[kPerm3[o][1]] &&
            mine[2] == theirs[kPerm3[o][2]])
          code = o;
      if (code < 0) throw std::runtime_error("face vertex mismatch");
      m.orient[q] = code;
    }

  // Geometric factors: A = [x_r x_s x_t] = [(v2-v1)/2 (v3-v1)/2 (v4-v1)/2], J = det A,
  // rows of A^-1 = (grad r, grad s, grad t) from the cofactors.
  m.geo.assign(size_t(K) * kGeoStride, 0.0);
  for (int k = 0; k < K; ++k) {
    const double* p[4];
    for (int v = 0; v < 4; ++v) p[v] = vxyz + 3 * size_t(m.etov[size_t(k) * 4 + v]);
    double xr[3], xs[3], xt[3];
    for (int d = 0; d < 3; ++d) {
      xr[d] = 0.5 * (p[1][d] - p[0][d]);
      xs[d] = 0.5 * (p[2][d] - p[0][d]);
      xt[d] = 0.5 * (p[3][d] - p[0][d]);
    }
    // cross products give the rows of the inverse scaled by J
    double cst[3] = {xs[1] * xt[2] - xs[2] * xt[1], xs[2] * xt[0] - xs[0] * xt[2], xs[0] * xt[1] - xs[1] * xt[0]};
    double ctr[3] = {xt[1] * xr[2] - xt[2] * xr[1], xt[2] * xr[0] - xt[0] * xr[2], xt[0] * xr[1] - xt[1] * xr[0]};
    double crs[3] = {xr[1] * xs[2] - xr[2] * xs[1], xr[2] * xs[0] - xr[0] * xs[2], xr[0] * xs[1] - xr[1] * xs[0]};
    double J = xr[0] * cst[0] + xr[1] * cst[1] + xr[2] * cst[2];
    if (!(J > 0.0)) throw std::runtime_error("non-positive Jacobian");
    double* g = &m.geo[size_t(k) * kGeoStride];
    for (int d = 0; d < 3; ++d) {
      g[0 + d] = cst[d] / J;  // grad r
      g[3 + d] = ctr[d] / J;  // grad s
      g[6 + d] = crs[d] / J;  // grad t
    }
    g[kGeoJ] = J;
    // outward normals: F1 -grad t, F2 -grad s, F3 grad r + grad s + grad t, F4 -grad r
    for (int f = 0; f < 4; ++f) {
      double nt[3];
      for (int d = 0; d < 3; ++d) {
        double gr = g[0 + d], gs = g[3 + d], gt = g[6 + d];
        nt[d] = (f == 0) ? -gt : (f == 1) ? -gs : (f == 2) ? (gr + gs + gt) : -gr;
      }
      double mag = std::sqrt(nt[0] * nt[0] + nt[1] * nt[1] + nt[2] * nt[2]);
      for (int d = 0; d < 3; ++d) g[kGeoNormal + 4 * f + d] = nt[d] / mag;
      g[kGeoNormal + 4 * f + 3] = mag;  // Fscale = sJ/J = |n~|
    }
  }

  // Physical node coordinates.
  const int Np = R.Np;
  m.x.assign(size_t(3) * K * Np, 0.0);
  for (int k = 0; k < K; ++k) {
    const double* p[4];
    for (int v = 0; v < 4; ++v) p[v] = vxyz + 3 * size_t(m.etov[size_t(k) * 4 + v]);
    for (int n = 0; n < Np; ++n) {
      double w[4] = {-(1.0 + R.r[n] + R.s[n] + R.t[n]), 1.0 + R.r[n], 1.0 + R.s[n], 1.0 + R.t[n]};
      for (int d = 0; d < 3; ++d)
        m.x[(size_t(d) * K + k) * Np + n] =
            0.5 * (w[0] * p[0][d] + w[1] * p[1][d] + w[2] * p[2][d] + w[3] * p[3][d]);
    }
  }

  // Locality order: elements sorted along a Morton curve through their centroids, so that
  // consecutive tiles are compact in space and most neighbour traces are read from nearby
  // memory (Sec. 5.3 lets the gather decide the element numbering).
  m.elem_of.resize(K);
  std::iota(m.elem_of.begin(), m.elem_of.end(), 0);
  if (reorder == 1) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    std::vector<std::array<double, 3>> cen(K);
    for (int k = 0; k < K; ++k)
      for (int d = 0; d < 3; ++d) {
        double c = 0;
        for (int v = 0; v < 4; ++v) c += vxyz[3 * size_t(m.etov[size_t(k) * 4 + v]) + d];
        cen[k][d] = 0.25 * c;
        lo[d] = std::min(lo[d], cen[k][d]);
        hi[d] = std::max(hi[d], cen[k][d]);
      }
    std::vector<uint64_t> code(K);
    for (int k = 0; k < K; ++k) {
      uint64_t c = 0;
      for (int d = 0; d < 3; ++d) {
        double span = hi[d] - lo[d];
        double u = span > 0 ? (cen[k][d] - lo[d]) / span : 0.0;
        uint64_t q = uint64_t(std::min(std::max(u, 0.0), 1.0) * double((1u << 21) - 1));
        c |= spread3(q) << d;
      }
      code[k] = c;
    }
    // with groups (the meshes of a batch) the order is by group first, so that each group
    // stays contiguous and its tiles hold only its own elements' neighbours
    std::stable_sort(m.elem_of.begin(), m.elem_of.end(), [&](int32_t a, int32_t b) {
      if (group && group[a] != group[b]) return group[a] < group[b];
      return code[a] < code[b];
    });
  } else if (reorder != 0) {
    throw std::runtime_error("unknown reorder mode");
  }
  m.pos_of.resize(K);
  for (int i = 0; i < K; ++i) m.pos_of[m.elem_of[i]] = i;

  m.face_code.resize(size_t(K) * 4);
  for (int i = 0; i < K; ++i) {
    int k = m.elem_of[i];
    for (int f = 0; f < 4; ++f) {
      size_t q = size_t(k) * 4 + f;
      int32_t code = kFacePec;
      if (m.orient[q] >= 0) {
        code = pack_face(m.pos_of[m.etoe[q]], m.orient[q], m.etof[q]);
      } else if (m.wall_kind[q] == 2) {
        code = kFaceAbsorbing;
      } else if (m.wall_kind[q] == 3) {
        code = kFaceScatter0 - int32_t(m.scat_face.size());
        m.scat_face.push_back(i * 4 + f);
      }
      m.face_code[size_t(i) * 4 + f] = code;
    }
  }
  return m;
}

std::vector<double> material_records(const MeshData& m, const double* eps, const double* mu) {
  const int K = m.K;
  std::vector<double> Z(K);
  for (int k = 0; k < K; ++k) {
    const double e = eps ? eps[k] : 1.0, u = mu ? mu[k] : 1.0;
    if (!(std::isfinite(e) && e > 0.0 && std::isfinite(u) && u > 0.0))
      throw std::runtime_error("eps and mu must be finite and positive");
    Z[k] = std::sqrt(u / e);
  }
  std::vector<double> rec(size_t(K) * kMatStride);
  for (int i = 0; i < K; ++i) {
    const int k = m.elem_of[i];
    const double e = eps ? eps[k] : 1.0, u = mu ? mu[k] : 1.0;
    double* r = &rec[size_t(i) * kMatStride];
    r[0] = 1.0 / e, r[1] = 1.0 / u, r[2] = e, r[3] = u;
    for (int f = 0; f < 4; ++f) {
      const size_t q = size_t(k) * 4 + f;
      const double fs = m.geo[size_t(k) * kGeoStride + kGeoNormal + 4 * f + 3];
      const double zm = Z[k], zp = m.orient[q] >= 0 ? Z[m.etoe[q]] : zm;
      const double ym = 1.0 / zm, yp = 1.0 / zp;
      r[kMatFace + 4 * f + 0] = fs / e * zp / (zm + zp);
      r[kMatFace + 4 * f + 1] = fs / e / (zm + zp);
      r[kMatFace + 4 * f + 2] = fs / u * yp / (ym + yp);
      r[kMatFace + 4 * f + 3] = fs / u / (ym + yp);
    }
  }
  return rec;
}

void canonical_maps(const RefOps& R, const MeshData& m, int32_t* vmapM, int32_t* vmapP) {
  const int Np = R.Np, Nfp = R.Nfp;
  for (int k = 0; k < m.K; ++k)
    for (int f = 0; f < 4; ++f) {
      size_t q = size_t(k) * 4 + f;
      for (int j = 0; j < Nfp; ++j) {
        size_t o = q * Nfp + j;
        vmapM[o] = k * Np + R.Fmask[f * Nfp + j];
        if (m.orient[q] < 0) {
          vmapP[o] = vmapM[o];
        } else {
          int f2 = m.etof[q];
          vmapP[o] = m.etoe[q] * Np + R.nbr_node[((size_t(f) * 4 + f2) * 6 + m.orient[q]) * Nfp + j];
        }
      }
    }
}

}  // namespace dgh

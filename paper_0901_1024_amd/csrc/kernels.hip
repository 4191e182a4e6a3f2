// Device kernels for the nodal DG Maxwell operator on gfx950 (MI355X).
//
// One workgroup owns a tile of consecutive elements (internal locality order) and computes,
// in one pass over HBM, every part of the semi-discrete operator of Sec. 2 (eq.
// semidiscrete-dg) for those elements:
//   - flux gather (Sec. 5.3): facial values of the element (from LDS) and of the neighbour
//     (from LDS when the neighbour is in the tile, else from global memory), upwind flux of
//     Sec. 6 or the perfectly conducting mirror state, scaled by Fscale = sJ/J;
//   - element-local differentiation (Sec. 5.4) with the per-element inverse-map
//     coefficients combined into the curl;
//   - flux lifting (Sec. 5.2) by the reference LIFT matrix;
//   - optionally the LSRK4 update (the "assembly" and RK steps of Sec. 6) fused as epilogue.
// Unlike the paper's split into separate grids, the tile keeps fields, face fluxes and the
// result on chip, so each field value crosses HBM once per stage.
#include <hip/hip_runtime.h>

#include "host/meshbuild.hpp"
#include "kernels.hpp"

namespace dgk {
namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

template <int N>
struct Dims {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int Nf4 = 4 * Nfp;
  static constexpr int E = (kThreads / Np) > 0 ? (kThreads / Np) : 1;
};

// Workgroups are dispatched round-robin over the XCDs; give every XCD a contiguous range of
// tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int per = nblocks / kXcds;
  return (bid % kXcds) * per + bid / kXcds;
}

template <typename T, int N, bool STAGE>
__global__ __launch_bounds__(kThreads) void stage_kernel(
    const T* __restrict__ u_in, T* __restrict__ out, T* __restrict__ res,
    const T* __restrict__ geo, const int32_t* __restrict__ fcode, const T* __restrict__ Dr,
    const T* __restrict__ Ds, const T* __restrict__ Dt, const T* __restrict__ LIFT,
    const int32_t* __restrict__ fmask, const int32_t* __restrict__ nbrnode, int K, int ntiles,
    T ca, T cb, T cdt) {
  using D = Dims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E;
  constexpr int G = dgh::kGeoStride;
  __shared__ T us[E * 6 * NP];
  __shared__ T fl[E * 6 * NF4];

  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntiles) return;
  const int base = tile * E;
  const int nel = min(E, K - base);

  // fields of the tile: contiguous in the element-major internal layout
  const T* src = u_in + size_t(base) * 6 * NP;
  for (int q = threadIdx.x; q < nel * 6 * NP; q += kThreads) us[q] = src[q];
  __syncthreads();

  // face fluxes, already multiplied by Fscale / 2 (the upwind flux carries a factor 1/2)
  for (int q = threadIdx.x; q < nel * NF4; q += kThreads) {
    const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
    const int elem = base + e;
    const T* g = geo + size_t(elem) * G + dgh::kGeoNormal + 4 * f;
    const T nx = g[0], ny = g[1], nz = g[2], hs = T(0.5) * g[3];
    const T* um = us + e * 6 * NP + fmask[f * NFP + j];
    const T Ex = um[0], Ey = um[NP], Ez = um[2 * NP], Hx = um[3 * NP], Hy = um[4 * NP], Hz = um[5 * NP];
    T dEx, dEy, dEz, dHx, dHy, dHz;
    const int code = fcode[size_t(elem) * 4 + f];
    if (code < 0) {  // perfectly conducting wall: E+ = -E-, H+ = H-
      dEx = T(-2) * Ex, dEy = T(-2) * Ey, dEz = T(-2) * Ez;
      dHx = dHy = dHz = T(0);
    } else {
      const int nb = code >> 5, o = (code >> 2) & 7, f2 = code & 3;
      const int nn = nbrnode[((f * 4 + f2) * 6 + o) * NFP + j];
      const int le = nb - base;
      const T* up = (le >= 0 && le < nel) ? us + le * 6 * NP + nn : u_in + size_t(nb) * 6 * NP + nn;
      dEx = up[0] - Ex, dEy = up[NP] - Ey, dEz = up[2 * NP] - Ez;
      dHx = up[3 * NP] - Hx, dHy = up[4 * NP] - Hy, dHz = up[5 * NP] - Hz;
    }
    const T ndE = nx * dEx + ny * dEy + nz * dEz;
    const T ndH = nx * dHx + ny * dHy + nz * dHz;
    T* o = fl + e * 6 * NF4 + fj;
    o[0 * NF4] = hs * (ny * dHz - nz * dHy + dEx - ndE * nx);
    o[1 * NF4] = hs * (nz * dHx - nx * dHz + dEy - ndE * ny);
    o[2 * NF4] = hs * (nx * dHy - ny * dHx + dEz - ndE * nz);
    o[3 * NF4] = hs * (nz * dEy - ny * dEz + dHx - ndH * nx);
    o[4 * NF4] = hs * (nx * dEz - nz * dEx + dHy - ndH * ny);
    o[5 * NF4] = hs * (ny * dEx - nx * dEy + dHz - ndH * nz);
  }
  __syncthreads();

  // one thread per (element, node): 18 reference derivatives, curl, lift, update
  for (int q = threadIdx.x; q < nel * NP; q += kThreads) {
    const int e = q / NP, n = q - e * NP;
    const int elem = base + e;
    const T* ue = us + e * 6 * NP;
    T ar[6], as[6], at[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) ar[c] = as[c] = at[c] = T(0);
    for (int j = 0; j < NP; ++j) {
      const T dr = Dr[n * NP + j], ds = Ds[n * NP + j], dt = Dt[n * NP + j];
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        const T v = ue[c * NP + j];
        ar[c] += dr * v;
        as[c] += ds * v;
        at[c] += dt * v;
      }
    }
    const T* g = geo + size_t(elem) * G;
    T dx[6], dy[6], dz[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      dx[c] = g[0] * ar[c] + g[3] * as[c] + g[6] * at[c];
      dy[c] = g[1] * ar[c] + g[4] * as[c] + g[7] * at[c];
      dz[c] = g[2] * ar[c] + g[5] * as[c] + g[8] * at[c];
    }
    T r[6];
    r[0] = dy[5] - dz[4];      // (curl H)_x
    r[1] = dz[3] - dx[5];      // (curl H)_y
    r[2] = dx[4] - dy[3];      // (curl H)_z
    r[3] = -(dy[2] - dz[1]);   // -(curl E)_x
    r[4] = -(dz[0] - dx[2]);   // -(curl E)_y
    r[5] = -(dx[1] - dy[0]);   // -(curl E)_z
    const T* fe = fl + e * 6 * NF4;
    for (int fj = 0; fj < NF4; ++fj) {
      const T l = LIFT[n * NF4 + fj];
#pragma unroll
      for (int c = 0; c < 6; ++c) r[c] += l * fe[c * NF4 + fj];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const size_t idx = (size_t(elem) * 6 + c) * NP + n;
      if (STAGE) {
        const T rv = ca * res[idx] + cdt * r[c];
        res[idx] = rv;
        out[idx] = ue[c * NP + n] + cb * rv;
      } else {
        out[idx] = r[c];
      }
    }
  }
}

template <typename T, int N>
hipError_t launch_stage_t(bool stage, const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = Dims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nblocks = ((ntiles + kXcds - 1) / kXcds) * kXcds;
  auto* u = static_cast<const T*>(a.u_in);
  auto* o = static_cast<T*>(a.out);
  auto* r = static_cast<T*>(a.res);
  auto* g = static_cast<const T*>(a.geo);
  auto* dr = static_cast<const T*>(ops.Dr);
  auto* ds = static_cast<const T*>(ops.Ds);
  auto* dt = static_cast<const T*>(ops.Dt);
  auto* lf = static_cast<const T*>(ops.LIFT);
  if (stage)
    stage_kernel<T, N, true><<<nblocks, kThreads, 0, s>>>(u, o, r, g, a.fcode, dr, ds, dt, lf, ops.fmask,
                                                         ops.nbrnode, a.K, ntiles, T(a.a), T(a.b), T(a.dt));
  else
    stage_kernel<T, N, false><<<nblocks, kThreads, 0, s>>>(u, o, r, g, a.fcode, dr, ds, dt, lf, ops.fmask,
                                                          ops.nbrnode, a.K, ntiles, T(0), T(0), T(0));
  return hipGetLastError();
}

template <typename T>
__global__ void to_internal_kernel(const T* __restrict__ canon, T* __restrict__ internal,
                                   const int32_t* __restrict__ elem_of, int K, int Np) {
  const int64_t total = int64_t(K) * 6 * Np;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * blockDim.x) {
    const int64_t i = q / (6 * Np);
    const int rem = int(q - i * 6 * Np);
    const int c = rem / Np, n = rem - c * Np;
    internal[q] = canon[(int64_t(c) * K + elem_of[i]) * Np + n];
  }
}

template <typename T>
__global__ void to_canonical_kernel(const T* __restrict__ internal, T* __restrict__ canon,
                                    const int32_t* __restrict__ pos_of, int K, int Np) {
  const int64_t total = int64_t(K) * 6 * Np;
  for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < total;
       q += int64_t(gridDim.x) * blockDim.x) {
    const int64_t c = q / (int64_t(K) * Np);
    const int64_t rem = q - c * K * Np;
    const int64_t k = rem / Np;
    const int n = int(rem - k * Np);
    canon[q] = internal[(int64_t(pos_of[k]) * 6 + c) * Np + n];
  }
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void energy_kernel(const T* __restrict__ u, const T* __restrict__ M,
                                                          const T* __restrict__ geo, int K,
                                                          double* __restrict__ partial) {
  constexpr int NP = Dims<N>::Np;
  __shared__ double red[kThreads];
  double acc = 0.0;
  const int e0 = blockIdx.x * kEnergyBlockElems;
  const int e1 = min(K, e0 + kEnergyBlockElems);
  for (int q = threadIdx.x; q < (e1 - e0) * NP; q += kThreads) {
    const int e = e0 + q / NP, i = q % NP;
    const T* ue = u + size_t(e) * 6 * NP;
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
      double mu = 0.0;
      for (int j = 0; j < NP; ++j) mu += double(M[i * NP + j]) * double(ue[c * NP + j]);
      s += mu * double(ue[c * NP + i]);
    }
    acc += 0.5 * double(geo[size_t(e) * dgh::kGeoStride + dgh::kGeoJ]) * s;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

template <typename T, int N>
hipError_t launch_energy_t(const void* u, const void* M, const void* geo, int K, double* partial,
                           hipStream_t s) {
  const int nb = (K + kEnergyBlockElems - 1) / kEnergyBlockElems;
  energy_kernel<T, N><<<nb, kThreads, 0, s>>>(static_cast<const T*>(u), static_cast<const T*>(M),
                                              static_cast<const T*>(geo), K, partial);
  return hipGetLastError();
}

template <typename T>
hipError_t dispatch_stage(int N, bool stage, const OpsView& o, const StageArgs& a, hipStream_t s) {
  switch (N) {
    case 1: return launch_stage_t<T, 1>(stage, o, a, s);
    case 2: return launch_stage_t<T, 2>(stage, o, a, s);
    case 3: return launch_stage_t<T, 3>(stage, o, a, s);
    case 4: return launch_stage_t<T, 4>(stage, o, a, s);
    case 5: return launch_stage_t<T, 5>(stage, o, a, s);
    case 6: return launch_stage_t<T, 6>(stage, o, a, s);
    case 7: return launch_stage_t<T, 7>(stage, o, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_energy(int N, const void* u, const void* M, const void* geo, int K, double* p,
                           hipStream_t s) {
  switch (N) {
    case 1: return launch_energy_t<T, 1>(u, M, geo, K, p, s);
    case 2: return launch_energy_t<T, 2>(u, M, geo, K, p, s);
    case 3: return launch_energy_t<T, 3>(u, M, geo, K, p, s);
    case 4: return launch_energy_t<T, 4>(u, M, geo, K, p, s);
    case 5: return launch_energy_t<T, 5>(u, M, geo, K, p, s);
    case 6: return launch_energy_t<T, 6>(u, M, geo, K, p, s);
    case 7: return launch_energy_t<T, 7>(u, M, geo, K, p, s);
  }
  return hipErrorInvalidValue;
}

int grid_for(int64_t total) {
  int64_t b = (total + kThreads - 1) / kThreads;
  return int(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace

int tile_elems(int N) {
  switch (N) {
    case 1: return Dims<1>::E;
    case 2: return Dims<2>::E;
    case 3: return Dims<3>::E;
    case 4: return Dims<4>::E;
    case 5: return Dims<5>::E;
    case 6: return Dims<6>::E;
    case 7: return Dims<7>::E;
  }
  return 0;
}

hipError_t launch_stage(int N, bool f64, bool stage, const OpsView& ops, const StageArgs& a,
                        hipStream_t s) {
  return f64 ? dispatch_stage<double>(N, stage, ops, a, s) : dispatch_stage<float>(N, stage, ops, a, s);
}

hipError_t launch_to_internal(bool f64, const void* canon, void* internal, const int32_t* elem_of,
                              int K, int Np, hipStream_t s) {
  const int g = grid_for(int64_t(K) * 6 * Np);
  if (f64)
    to_internal_kernel<double><<<g, kThreads, 0, s>>>(static_cast<const double*>(canon),
                                                      static_cast<double*>(internal), elem_of, K, Np);
  else
    to_internal_kernel<float><<<g, kThreads, 0, s>>>(static_cast<const float*>(canon),
                                                     static_cast<float*>(internal), elem_of, K, Np);
  return hipGetLastError();
}

hipError_t launch_to_canonical(bool f64, const void* internal, void* canon, const int32_t* pos_of,
                               int K, int Np, hipStream_t s) {
  const int g = grid_for(int64_t(K) * 6 * Np);
  if (f64)
    to_canonical_kernel<double><<<g, kThreads, 0, s>>>(static_cast<const double*>(internal),
                                                       static_cast<double*>(canon), pos_of, K, Np);
  else
    to_canonical_kernel<float><<<g, kThreads, 0, s>>>(static_cast<const float*>(internal),
                                                      static_cast<float*>(canon), pos_of, K, Np);
  return hipGetLastError();
}

hipError_t launch_energy(int N, bool f64, const void* u, const void* M, const void* geo, int K,
                         double* partial, hipStream_t s) {
  return f64 ? dispatch_energy<double>(N, u, M, geo, K, partial, s)
             : dispatch_energy<float>(N, u, M, geo, K, partial, s);
}

}  // namespace dgk

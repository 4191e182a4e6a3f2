// Launch interface of the device kernels (used by the C ABI layer).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace dgk {

// Device views of the per-handle constant data.
struct OpsView {
  const void* Dr;
  const void* Ds;
  const void* Dt;
  const void* LIFT;
  const void* M;
  const int32_t* fmask;    // 4 x Nfp
  const int32_t* nbrnode;  // 4 x 4 x 6 x Nfp
  // The concatenated operator OpCat = [Dr | Ds | Dt | LIFT] (Np x KD, each D block
  // zero-padded to roundup(Np, 4) columns, KD = 3 roundup(Np, 4) + 4 Nfp) in MFMA fragment
  // order (FP32 contraction kernels only; NULL where unused):
  //   [nt][kk][lane] = OpCat[16 nt + lane % 16][4 kk + lane / 16]  for the full 16-node tiles,
  //   then [k][c]    = OpCat[16 NT + c][k] (zero for rows >= Np)    for the remaining nodes.
  const void* opfrag;
};

// Floats in the fragment-ordered operator for order N (0 when no contraction kernel serves N).
int opcat_words(int N);
// Whether the FP32 MFMA stage kernel serves order N.
bool mfma_order(int N);

struct StageArgs {
  const void* u_in;  // internal layout [K][6][Np]
  void* out;         // rhs (RHS mode) or u_out (stage mode), internal layout
  void* res;         // RK residual, internal layout (stage mode only)
  const void* geo;   // [K][26]
  const int32_t* fcode;  // [K][4]
  int K;
  double a, b, dt;   // stage coefficients (stage mode only)
};

// Elements per workgroup tile of the stage kernel for order N.
int tile_elems(int N);

// One RHS evaluation (stage == false) or one fused LSRK4 stage (stage == true).
hipError_t launch_stage(int N, bool f64, bool stage, const OpsView& ops, const StageArgs& a,
                        hipStream_t s);

// Canonical [6][K][Np] <-> internal [K][6][Np] (internal position i holds user element
// elem_of[i]).
hipError_t launch_to_internal(bool f64, const void* canon, void* internal, const int32_t* elem_of,
                              int K, int Np, hipStream_t s);
hipError_t launch_to_canonical(bool f64, const void* internal, void* canon, const int32_t* pos_of,
                               int K, int Np, hipStream_t s);

// Partial energies: one double per block of `energy_block_elems` elements written to
// `partial`; the caller sums them.
constexpr int kEnergyBlockElems = 64;
hipError_t launch_energy(int N, bool f64, const void* u, const void* M, const void* geo, int K,
                         double* partial, hipStream_t s);

}  // namespace dgk

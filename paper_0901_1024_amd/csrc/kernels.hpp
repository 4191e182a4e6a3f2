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
  // The concatenated operator OpCat = [Dr | Ds | Dt | LIFT] (each D block zero-padded to
  // roundup(Np, 4) columns, LIFT to roundup(4 Nfp, 16)) in the fragment order of the FP32
  // contraction kernel (NULL where unused); opfrag_source() says which entry each word holds.
  const void* opfrag;
};

// Words in the fragment-ordered operator for order N in the given precision (0 when no
// contraction kernel serves N). The layouts of the two precisions agree except at N = 4, where
// the FP32 kernel has two column tiles and a 4-column tail and the FP64 one three column tiles.
int opcat_words(int N, bool f64);
// Whether the FP32 MFMA stage kernel serves order N.
bool mfma_order(int N);
// Whether an FP64 MFMA stage kernel serves order N (N = 3..7; each reads the operator table of
// the FP32 kernel of the same order in FP64, except at N = 4: see opcat_words).
bool dmfma_order(int N);
// Whether the split-BF16 contraction kernel serves order N.
bool bf16x3_order(int N);
// 16-bit words of its operator table (high and low bf16 parts in lane order).
int bopcat_words(int N);
// Word w of that table holds part `part` (0 high, 1 low) of row n of operator block blk
// (0, 1, 2 = Dr, Ds, Dt; 3 = LIFT) at column col; zero when n or col fall outside the operator
// (n >= Np, col >= Np for a D block, col >= 4 Nfp for LIFT).
void bopfrag_source(int N, int w, int* n, int* blk, int* col, int* part);
// Words per (element, field) row of the internal field arrays, [K][6][S]: Np, rounded up to a
// multiple of 4 for the FP32 contraction orders (the pad words are kept zero).
int row_stride(int N, bool f64);
// Word w of the fragment-ordered operator of order N (in the layout of the given precision)
// holds row n of operator block blk (0, 1, 2 = Dr, Ds, Dt; 3 = LIFT) at column col; it is zero
// when n, col fall outside the operator (n >= Np, col >= Np for a D block, col >= 4 Nfp for
// LIFT).
void opfrag_source(int N, bool f64, int w, int* n, int* blk, int* col);

// Incident field of the scattered-field form (read on scatterer faces only).
struct SrcArgs {
  const double* rec = nullptr;    // p (3), profile c0..c4 (5), time at the start of the step (1);
                                  // NULL when the mesh has no scatterer faces
  const double* phase = nullptr;  // k.x at the face nodes of scatterer face i: [i][Nfp]
  double toff = 0.0;              // this stage's time minus the step's start time (c_i dt)
};
// Words of the incident record.
constexpr int kSrcRecWords = 9;

struct StageArgs {
  const void* u_in;  // internal layout [K][6][S], S = row_stride(N, f64)
  void* out;         // rhs (RHS mode) or u_out (stage mode), internal layout
  void* res;         // RK residual, internal layout (stage mode only)
  const void* geo;   // [K][26]
  const int32_t* fcode;  // [K][4]
  const void* mat;   // [K][20] material records of a heterogeneous medium, or NULL (vacuum)
  int K;
  double a, b, dt;   // stage coefficients (stage mode only)
  SrcArgs src;       // scattered-field form (src.rec == NULL: none)
  bool split_bf16 = false;   // FP32 state, split-BF16 contraction (operator table in bf16)
  bool wide_tiles = false;   // FP32 N = 3: the 16-element contraction kernel instead of the 8-element one
};

// One RHS evaluation (stage == false) or one fused LSRK4 stage (stage == true).
hipError_t launch_stage(int N, bool f64, bool stage, const OpsView& ops, const StageArgs& a,
                        hipStream_t s);

// Canonical [6][K][Np] <-> internal [K][6][S] (user element e sits at internal position
// pos_of[e]; to_internal writes the pad words as zero).
hipError_t launch_to_internal(int N, bool f64, const void* canon, void* internal, const int32_t* pos_of,
                              int K, hipStream_t s);
hipError_t launch_to_canonical(int N, bool f64, const void* internal, void* canon, const int32_t* pos_of,
                               int K, hipStream_t s);

// Zero `bytes` bytes at p (16-byte aligned) with a kernel: a memset node recorded into a graph
// that a caller captures has given wrong results on replay, a kernel node has not.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

// Advance the step's start time in the incident record by dt (after the fifth stage).
hipError_t launch_advance_clock(double* rec, double dt, hipStream_t s);
// Set the step's start time in the incident record.
hipError_t launch_set_clock(double* rec, double t, hipStream_t s);

// Partial energies: one double per block of `energy_block_elems` elements written to
// `partial`; the caller sums them.
constexpr int kEnergyBlockElems = 64;
hipError_t launch_energy(int N, bool f64, const void* u, const void* M, const void* geo, const void* mat,
                         int K, double* partial, hipStream_t s);

// out[0] = sum of partial[0 .. n-1] (device pointers), by one workgroup in a fixed order.
hipError_t launch_sum(const double* partial, int n, double* out, hipStream_t s);

// The allocation-free energy call keeps its partial sums in a static device array of
// kNoallocPartials doubles (512 KiB per device, so K <= kNoallocPartials * kEnergyBlockElems).
constexpr int kNoallocPartials = 65536;
// Looks up the device address of that array on `device` once (hipGetSymbolAddress with the
// device current); later calls return at once. Thread-safe.
hipError_t noalloc_scratch_init(int device);
// The address found by noalloc_scratch_init on `device`, or NULL before it.
double* noalloc_scratch(int device);

}  // namespace dgk

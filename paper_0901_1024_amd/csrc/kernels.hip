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

#include <atomic>
#include <cstdint>
#include <mutex>

#include "host/meshbuild.hpp"
#include "kernels.hpp"

// Device scratch of the allocation-free energy call: one partial sum per block of elements.
// Each device holds its own copy for the life of the process; host code must use the address
// returned by hipGetSymbolAddress on that device (noalloc_scratch), never this name.
static __device__ __align__(256) double scratch[dgk::kNoallocPartials];

namespace dgk {
namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;
constexpr int kMaxDevices = 64;

template <int N>
struct Dims {
  static constexpr int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  static constexpr int Nfp = (N + 1) * (N + 2) / 2;
  static constexpr int Nf4 = 4 * Nfp;
  static constexpr int E = (kThreads / Np) > 0 ? (kThreads / Np) : 1;
};

// Words per (element, field) row of the internal field arrays [K][6][S]: Np, padded to a
// multiple of 4 (pad words zero) for the orders that the FP32 contraction kernels serve, so
// that their tiles move in aligned 16-byte chunks.
constexpr bool contraction_order(int N) { return N >= 3 && N <= 7; }
template <typename T, int N>
constexpr int kRowStride = (sizeof(T) == 4 && contraction_order(N)) ? (Dims<N>::Np + 3) / 4 * 4 : Dims<N>::Np;

// Jump u+ - u- at a face node (Sec. 6): a perfectly conducting wall mirrors the interior
// state (E+ = -E-, H+ = H-), an absorbing face has zero exterior state, an interior face
// takes the neighbour's trace p (six fields).
template <typename T>
__device__ __forceinline__ void face_jump(int code, const T (&m)[6], const T (&p)[6], T (&d)[6]) {
  // a scatterer face is a wall for the total field: m carries E- + E_inc there
  const bool inner = code >= 0, pec = code == dgh::kFacePec || code <= dgh::kFaceScatter0;
#pragma unroll
  for (int c = 0; c < 6; ++c) {   // selects, no branches
    const T wall = pec ? (c < 3 ? T(-2) * m[c] : T(0)) : -m[c];
    d[c] = inner ? p[c] - m[c] : wall;
  }
}

// Scattered-field form: add the incident plane wave E_inc = p f(k.x - t) to the interior E at
// face node j of scatterer face `code` (<= kFaceScatter0), so that face_jump mirrors the total
// field. f(s) = c0 + c1 s + c2 sin(c3 s + c4), t = step start + stage offset; evaluated in
// double for either working precision.
template <typename T>
__device__ __forceinline__ void add_incident(const SrcArgs& src, int code, int j, int nfp, T (&m)[6]) {
  const double* r = src.rec;
  const double ph = src.phase[size_t(dgh::kFaceScatter0 - code) * nfp + j];
  const double x = ph - (r[8] + src.toff);
  const double f = r[3] + r[4] * x + r[5] * sin(r[6] * x + r[7]);
  m[0] += T(r[0] * f);
  m[1] += T(r[1] * f);
  m[2] += T(r[2] * f);
}

// Upwind flux of Sec. 6 at a face node with unit normal n and jump d = (dE, dH), written to
// o[0], o[os], ..., o[5 os] already scaled: in vacuum by hs = Fscale / 2; in a medium by the
// impedance weights w = (A, B, C, D) of the material record, which fold in Fscale, 1/eps, 1/mu.
template <typename T>
__device__ __forceinline__ void upwind_flux(bool medium, T nx, T ny, T nz, T hs, const T (&w)[4],
                                            const T (&d)[6], T* o, int os) {
  const T dEx = d[0], dEy = d[1], dEz = d[2], dHx = d[3], dHy = d[4], dHz = d[5];
  const T ndE = nx * dEx + ny * dEy + nz * dEz;
  const T ndH = nx * dHx + ny * dHy + nz * dHz;
  if (medium) {
    const T A = w[0], B = w[1], C = w[2], Dd = w[3];
    o[0 * os] = A * (ny * dHz - nz * dHy) + B * (dEx - ndE * nx);
    o[1 * os] = A * (nz * dHx - nx * dHz) + B * (dEy - ndE * ny);
    o[2 * os] = A * (nx * dHy - ny * dHx) + B * (dEz - ndE * nz);
    o[3 * os] = C * (nz * dEy - ny * dEz) + Dd * (dHx - ndH * nx);
    o[4 * os] = C * (nx * dEz - nz * dEx) + Dd * (dHy - ndH * ny);
    o[5 * os] = C * (ny * dEx - nx * dEy) + Dd * (dHz - ndH * nz);
  } else {
    o[0 * os] = hs * (ny * dHz - nz * dHy + dEx - ndE * nx);
    o[1 * os] = hs * (nz * dHx - nx * dHz + dEy - ndE * ny);
    o[2 * os] = hs * (nx * dHy - ny * dHx + dEz - ndE * nz);
    o[3 * os] = hs * (nz * dEy - ny * dEz + dHx - ndH * nx);
    o[4 * os] = hs * (nx * dEz - nz * dEx + dHy - ndH * ny);
    o[5 * os] = hs * (ny * dEx - nx * dEy + dHz - ndH * nz);
  }
}

// Workgroups are dispatched round-robin over the XCDs; give every XCD a contiguous range of
// tiles so that neighbouring tiles share an L2.
__device__ __forceinline__ int xcd_tile(int bid, int nblocks) {
  const int per = nblocks / kXcds;
  return (bid % kXcds) * per + bid / kXcds;
}

template <typename T, int N, bool STAGE>
__global__ __launch_bounds__(kThreads) void stage_kernel(
    const T* __restrict__ u_in, T* __restrict__ out, T* __restrict__ res,
    const T* __restrict__ geo, const int32_t* __restrict__ fcode, const T* __restrict__ mat,
    const T* __restrict__ Dr, const T* __restrict__ Ds, const T* __restrict__ Dt,
    const T* __restrict__ LIFT, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, T ca, T cb, T cdt, SrcArgs inc) {
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

  // face fluxes, already multiplied by Fscale / 2 (the upwind flux carries a factor 1/2), or
  // in a heterogeneous medium by the folded impedance weights of the material record
  for (int q = threadIdx.x; q < nel * NF4; q += kThreads) {
    const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
    const int elem = base + e;
    const T* g = geo + size_t(elem) * G + dgh::kGeoNormal + 4 * f;
    const T nx = g[0], ny = g[1], nz = g[2], hs = T(0.5) * g[3];
    const T* um = us + e * 6 * NP + fmask[f * NFP + j];
    T m[6], p[6] = {}, d[6], w[4] = {};
    for (int c = 0; c < 6; ++c) m[c] = um[c * NP];
    const int code = fcode[size_t(elem) * 4 + f];
    if (code >= 0) {
      const int nb = code >> 5, o = (code >> 2) & 7, f2 = code & 3;
      const int nn = nbrnode[((f * 4 + f2) * 6 + o) * NFP + j];
      const int le = nb - base;
      const T* up = (le >= 0 && le < nel) ? us + le * 6 * NP + nn : u_in + size_t(nb) * 6 * NP + nn;
      for (int c = 0; c < 6; ++c) p[c] = up[c * NP];
    }
    if (inc.rec && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
    face_jump(code, m, p, d);
    if (mat) {
      const T* mw = mat + size_t(elem) * dgh::kMatStride + dgh::kMatFace + 4 * f;
      for (int c = 0; c < 4; ++c) w[c] = mw[c];
    }
    upwind_flux(mat != nullptr, nx, ny, nz, hs, w, d, fl + e * 6 * NF4 + fj, NF4);
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
    if (mat) {                 // 1/eps, 1/mu (the lifted fluxes carry them already)
      const T ie = mat[size_t(elem) * dgh::kMatStride], im = mat[size_t(elem) * dgh::kMatStride + 1];
      r[0] *= ie, r[1] *= ie, r[2] *= ie, r[3] *= im, r[4] *= im, r[5] *= im;
    }
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

// ---------------------------------------------------------------------------------------
// MFMA form of the fused stage (FP32).
//
// Because the inverse-map derivatives are constant per element, the curl can be taken before
// differentiating (the freedom to commute F(u) with the local differentiation noted in
// Sec. 4): with c[mu][nu] = d r_mu / d x_nu,
//   (curl H)_a = sum_mu D_mu (c[mu][b] H_c - c[mu][c] H_b),  (a,b,c) cyclic,
// and likewise -(curl E)_a. Volume and surface terms then form one contraction per element
// and field:  rhs = [Dr | Ds | Dt | LIFT] * [G_r; G_s; G_t; Fscale/2 * flux],
// an (Np x KD) operator times a (KD x 6E) operand, for a tile of E elements.
//
// Orientation: rows = (field, element) pairs, columns = nodes, so each result row lands on
// consecutive nodes. Full 16-node column tiles run on v_mfma_f32_16x16x4f32. The remaining
// Np mod 16 columns ride along on v_mfma_f32_4x4x1f32 fed with the same operand registers:
// its 16 blocks are read as (k-group g, row quad) pairs, so lane (row, g) supplies the value
// it already holds for the 16x16x4 step, the tail operator supplies column c of k-group g,
// and a sum over the four k-groups (cross-lane) finishes the tail. The volume part of the
// operand is formed on the fly from the field tile in LDS, whose rows are padded to a
// multiple of 4 nodes; the face part (Fscale/2 * flux) is materialised in LDS. Every operand
// and operator read is a 16-byte LDS read that feeds four k-steps, so the contraction issues
// few LDS instructions and waits.
//
// k-steps of the 16x16x4 contraction (lane group g = lane / 16 holds k-index g of each step):
//   volume quads  (jb, mu), jb < NPP / 16:  4 steps, group g at column 16 jb + 4 g + s of D_mu;
//   face quads    fb < NF / 16:             4 steps, group g at face column 16 fb + 4 g + s;
//   volume singles (r, mu), r < VR:         1 step,  group g at column 16 VB + 4 r + g of D_mu.
// A quad's four fragments sit in one float4 per lane; singles are one float per lane.

template <int N>
struct MDims {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, Nf4 = Dims<N>::Nf4;
  static constexpr int E = 16;                       // elements per tile
  static constexpr int ROWS = 6 * E;                 // (field, element) rows, field-major
  static constexpr int NPP = (Np + 3) / 4 * 4;       // volume block per direction, padded
  static constexpr int ES = 6 * NPP + 4;             // element stride of the padded tile (= 4 mod 8)
  static constexpr int PC = NPP / 4;                 // 16-byte chunks per padded row
  static constexpr int LAST = Np - 4 * (PC - 1);     // field words in the last chunk of a row
  static constexpr int TC = 6 * E * PC;              // chunks per tile
  static constexpr int CPC = (TC + kThreads - 1) / kThreads;   // chunks per thread
  // per-wave issue priorities (contraction first); at N = 3 the stage is bound by its memory
  // phases, and serving the short contraction first slows it (313 against 286 us per stage)
  static constexpr bool PRIO = N >= 4;
  // waves per SIMD the register budget is set for: four at N = 3 (128 VGPRs, a few spills, four
  // workgroups per CU: 274 against 289 us per stage), two at N = 4
  static constexpr int WPE = N == 3 ? 4 : 2;
  static_assert(ES % 4 == 0, "element rows of the padded tile are 16-byte aligned");
  static constexpr int NF = (Nf4 + 15) / 16 * 16;    // face block, padded
  static constexpr int RSL = NF + 4;                 // flux row stride (= 4 mod 8)
  static constexpr int KV = 3 * NPP;                 // volume part of the contraction
  static constexpr int KD = KV + NF;                 // contraction length
  static constexpr int KS = KD / 4;                  // k-steps
  static constexpr int VB = NPP / 16;                // full 16-column volume blocks
  static constexpr int VR = (NPP - 16 * VB) / 4;     // single steps per direction
  static constexpr int QV = 3 * VB, QF = NF / 16;    // volume and face quads
  static constexpr int NQ = QV + QF;
  static constexpr int NT = Np / 16;                 // full 16-node column tiles
  static constexpr int TAIL = Np - 16 * NT;          // columns left for the 4x4 blocks
  static constexpr int RT = ROWS / 16;               // 16-row tiles (one field each)
  static constexpr int TILES = RT * NT;              // dealt round-robin to the four waves
  static constexpr int TPW = (TILES + 3) / 4;
  static constexpr int FIT = (E * Nf4 + kThreads - 1) / kThreads;  // face nodes per thread
  // fragment-ordered operator: per column tile NQ float4 quads then 3 VR singles per lane;
  // then the tail columns, per quad [g][c][4 steps], per single [g][c]
  static constexpr int OPC = NT * KS * 64 + KS * 16;
  static_assert(4 * NQ + 3 * VR == KS, "k-steps are quads and singles");
  static_assert(NT == 1 || NT == 2 || NT == 4, "a wave's tiles must share one column tile");
  static_assert(TAIL <= 4, "the tail is one 4-column block");
  // after the contraction the flux rows are free for the rhs staging (laid out like up_s)
  static_assert(E * ES <= ROWS * RSL, "staging must fit in the flux rows");
};

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned uint4v __attribute__((ext_vector_type(4)));
constexpr int kNonTemporal = 2;   // cache policy of a buffer access: nontemporal

// Resource for raw buffer accesses to the nbytes at base (word 3 in the gfx9 layout: 32-bit data
// format). A lane whose byte offset lies at or past nbytes is not stored (range check), so a
// store can be issued by every lane with no condition.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(void* base, int nbytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, 0, nbytes, 0x00020000);
}

// MAT: heterogeneous medium. 1/eps and 1/mu of the tile's elements ride in the unused last
// words of each element row of the padded tile (up_s) and scale the operand coefficients;
// the face weights of the material records are prefetched with the tile into LDS (wmat).
template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MDims<N>::WPE, MDims<N>::WPE))) void mfma_stage_kernel(
    const float* __restrict__ u_in, float* __restrict__ out, float* __restrict__ res,
    const float* __restrict__ geo, const int32_t* __restrict__ fcode, const float* __restrict__ mat,
    const float* __restrict__ opf, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, float ca, float cb, float cdt, SrcArgs inc) {
  using D = MDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES,
                NF = D::NF, KS = D::KS, RSL = D::RSL, NT = D::NT,
                TAIL = D::TAIL, TILES = D::TILES, TPW = D::TPW, FIT = D::FIT, PC = D::PC,
                LAST = D::LAST, TC = D::TC, CPC = D::CPC, VB = D::VB, VR = D::VR, QV = D::QV,
                QF = D::QF, NQ = D::NQ;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;                                   // words of geometry per tile
  constexpr int GPT = (GW + kThreads - 1) / kThreads;
  // field tile [e][f][NPP]: rows padded to NPP words (pad columns zero), element stride ES
  __shared__ __align__(16) float up_s[E * ES];
  __shared__ __align__(16) float gl[D::ROWS * RSL];   // Fscale/2 * flux [f E + e][fj]; later staging
  __shared__ __align__(16) float bfs[NT * KS * 64];   // operator fragments
  __shared__ __align__(16) float tops[TAIL > 0 ? KS * 16 : 4];  // tail operator fragments
  __shared__ float gt[GW];                            // geometric records of the tile
  __shared__ __align__(16) float wmat[MAT ? E * 4 * dgh::kMatFace : 4];   // MAT: [e][f][A B C D]
  __shared__ int32_t fcb[2][E * 4];                   // face records: this tile, the next
  __shared__ uint8_t nbr_s[96 * NFP];                 // neighbour node table
  __shared__ uint8_t fm_s[4 * NFP];                   // face node lists

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, in an SGPR
  const int g4 = lane >> 4, li = lane & 15;
  // The field arrays hold rows of NPP words (pad words zero), [K][6][NPP]: word q of a tile
  // sits at slot(q) of up_s, whose element rows are ES apart. Chunk c (16 bytes) of a tile is
  // aligned both in the arrays (words 4c ..) and in up_s (slot(4c) ..).
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NPP);
    return e * ES + (q - e * 6 * NPP);
  };
  // zero the pad words of the last chunk of a row (they carry no node)
  auto pad_zero = [](int c, floatx4 v) __attribute__((always_inline)) {
    if (LAST < 4 && c % PC == PC - 1) {
      if (LAST <= 3) v.w = 0.f;
      if (LAST <= 2) v.z = 0.f;
      if (LAST <= 1) v.y = 0.f;
    }
    return v;
  };

  // Persistent schedule: workgroups are dispatched round-robin over the XCDs; XCD x owns the
  // contiguous tile range [x TX, (x+1) TX) and its workgroups sweep it together, so at any time
  // an XCD works on one window of neighbouring tiles (shared L2 for the neighbour traces).
  const int nwg = gridDim.x / kXcds;                 // workgroups per XCD (grid is a multiple of 8)
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  // once per workgroup: operator fragments, node tables, tail operator, zero padding
  const int nt = wave % NT;
  for (int q = tid; q < NT * KS * 64; q += kThreads) bfs[q] = opf[q];
  for (int q = tid; q < 96 * NFP; q += kThreads) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += kThreads) fm_s[q] = uint8_t(fmask[q]);
  if (TAIL > 0)
    for (int q = tid; q < KS * 16; q += kThreads) tops[q] = opf[NT * KS * 64 + q];
  // up_s starts zeroed, so that the rows past the elements of a ragged tile hold finite values
  for (int q = tid; q < E * ES; q += kThreads) up_s[q] = 0.f;
  __syncthreads();

  // Prefetch registers: fields and geometry of the next tile, the neighbour traces of its
  // face nodes, and the face records of the tile after it. In the material variant the
  // face-node slot of this thread is made opaque so that its index arithmetic is not hoisted
  // out of the tile loop.
  int tq = tid;
  if (MAT) asm volatile("" : "+v"(tq));
  floatx4 pu[CPC];
  float pg[GPT];
  float nup[FIT][6];   // exterior traces u+ of the face nodes tq + r kThreads (all six fields)
  int32_t pf = 0;
  float pm = 0.f, pw = 0.f;   // MAT: 1/eps (even threads) or 1/mu (odd threads) of element tid / 2
  // Every thread loads every slot, on every path, its index clamped into its array (a missing
  // next tile, and the part of a ragged one past the end of the arrays, loads values that are
  // not used; below the end the clamped index is the right one): an exec-masked load makes the
  // compiler wait for all outstanding loads before reusing its registers, and a load skipped
  // on some path makes a later wait for one load fall back to waiting for all of them.
  const size_t fc_last = size_t(K) * 4 - 1;
  const size_t chunk_last = size_t(K) * 6 * NPP / 4 - 1;
  const floatx4* u4 = reinterpret_cast<const floatx4*>(u_in);
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int j = 0; j < CPC; ++j) pu[j] = u4[min(size_t(t) * TC + min(tid + j * kThreads, TC - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * kThreads, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);   // word qw % 16 of the face weights of element qw / 16
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  // neighbour traces of tile t (face-node slots r0 .. r1 - 1 of this thread) from its face
  // records fcv (wall and absorbing faces, and slots past the tile, read their own element:
  // the values are not used)
  auto gather = [&](int t, const int32_t* fcv, int r0, int r1) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = r0; r < r1; ++r) {
      const int q = min(tq + r * kThreads, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const float* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NPP + nn : size_t(e0 + e) * 6 * NPP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NPP];
    }
  };
  int par = 0;   // fcb[par]: face records of this tile; fcb[par ^ 1]: of the next one
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  gather(tile, fcb[0], 0, FIT);
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  // The first tile's loads complete here, once per workgroup: nothing issued before the loop is
  // then pending at its head, and the compiler counts each wait inside the loop from the loop's
  // own order of issue (loads, then the write-out stores) instead of the prologue's.
  __builtin_amdgcn_s_waitcnt(0);

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    // the tile whose loads are issued during this one (this tile again when it is the last)
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;
    const size_t tb = size_t(base) * 6 * NPP;

    // ---- tile into LDS (from the prefetch registers when full), one aligned 16-byte write
    // per chunk. The chunk index is made opaque per tile so that its slot arithmetic is
    // recomputed rather than kept live.
    int tz = tid;
    asm volatile("" : "+v"(tz));
    if (full) {
#pragma unroll
      for (int j = 0; j < CPC; ++j) {
        const int c = tz + j * kThreads;
        if ((j + 1) * kThreads <= TC || c < TC) *reinterpret_cast<floatx4*>(up_s + slot(4 * c)) = pu[j];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * kThreads;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      // a ragged tile comes from the prefetch registers too: the clamped loads read the right
      // words below the end of the arrays (no load on this path)
      const int nc = nel * 6 * NPP / 4;
#pragma unroll
      for (int j = 0; j < CPC; ++j) {
        const int c = tz + j * kThreads;
        if (c < nc) *reinterpret_cast<floatx4*>(up_s + slot(4 * c)) = pu[j];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * kThreads;
        if (q < nel * G) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * nel) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * nel) wmat[tid] = pw;
    }
    __syncthreads();

    floatx4 rs[CPC];

    // Issue priority (per wave): the two workgroups on a CU interleave their phases on each
    // SIMD; the wave in its contraction is served first so that the matrix pipe stays fed,
    // then a wave in its flux phase, which the contraction waits for; the loads, staging and
    // write-out fill the gaps.
    if (D::PRIO) __builtin_amdgcn_s_setprio(2);
    // ---- face fluxes from the exterior traces gathered during the previous tile
    const int32_t* fc = fcb[par];
    {
      floatx4 wm[FIT];   // MAT: face weights A B C D
      if (MAT) {
#pragma unroll
        for (int r = 0; r < FIT; ++r) {
          const int q = min(tq + r * kThreads, nel * NF4 - 1);
          const int e = q / NF4, f = (q - e * NF4) / NFP;
          wm[r] = *reinterpret_cast<const floatx4*>(wmat + 16 * e + 4 * f);
        }
      }
      // face columns NF4 .. NF-1 of every row are padding: keep them zero
      if constexpr (NF > NF4)
        for (int q = tid; q < D::ROWS * (NF - NF4); q += kThreads) {
          const int row = q / (NF - NF4);
          gl[row * RSL + NF4 + (q - row * (NF - NF4))] = 0.f;
        }
#pragma unroll
      for (int r = 0; r < FIT; ++r) {
        const int q = tq + r * kThreads;
        if (q < nel * NF4) {
          const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
          const float* g = gt + e * G + dgh::kGeoNormal + 4 * f;
          const float nx = g[0], ny = g[1], nz = g[2], hs = 0.5f * g[3];
          const float* um = up_s + e * ES + fm_s[f * NFP + j];
          float m[6], d[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) m[c] = um[c * NPP];
          const int code = fc[e * 4 + f];
          if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
          face_jump(code, m, nup[r], d);
          const float w[4] = {wm[r].x, wm[r].y, wm[r].z, wm[r].w};
          upwind_flux(MAT, nx, ny, nz, hs, w, d, gl + e * RSL + fj, E * RSL);
        }
      }
    }
    __syncthreads();
    if (STAGE) {
#pragma unroll
      for (int j = 0; j < CPC; ++j)   // clamped like the prefetch (right below the end of the array)
        rs[j] = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(res) +
                                           min(size_t(tile) * TC + min(tid + j * kThreads, TC - 1), chunk_last));
    }

    if (D::PRIO) __builtin_amdgcn_s_setprio(3);
    // ---- main contraction: tiles wave, wave + 4, ... (row tile = field, lane row = element li).
    // A wave with fewer than TPW tiles repeats its last one and drops the result (branch-free).
    // The tail columns accumulate in tacc on the waves of column tile 0 only (a wave-uniform
    // condition: the other waves would drop them).
    floatx4 acc[TPW], tacc[TPW];
    {
      float pc[TPW][3], qc[TPW][3];   // operand = pc[mu] * V_c[j] + qc[mu] * V_b[j]
      const float* vc[TPW];
      const float* vb[TPW];
      const float* fl[TPW];
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
        acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        tacc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int tt = min(wave + 4 * t, TILES - 1);
        const int f = tt / NT;
        const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
        const int srcf = f < 3 ? 3 : 0;            // H feeds the E rows, E the H rows
        const float sg = f < 3 ? 1.f : -1.f;
        const float* cm = gt + li * G;
        // MAT: 1/eps on the E rows, 1/mu on the H rows
        const float sm = MAT ? sg * up_s[li * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          pc[t][mu] = sm * cm[3 * mu + b];
          qc[t][mu] = -sm * cm[3 * mu + c];
        }
        vc[t] = up_s + li * ES + (srcf + c) * NPP;
        vb[t] = up_s + li * ES + (srcf + b) * NPP;
        fl[t] = gl + (f * E + li) * RSL + 4 * g4;
      }
      const floatx4* bq = reinterpret_cast<const floatx4*>(bfs + nt * KS * 64) + lane;   // quads
      const float* bs = bfs + nt * KS * 64 + NQ * 256 + lane;                         // singles
      const int tl = 4 * g4 + (li & 3);   // tail fragment slot: k-group g4, column li mod 4
      const floatx4* tq = reinterpret_cast<const floatx4*>(tops) + tl;
      const float* ts = tops + NQ * 64 + tl;
#pragma unroll
      for (int jb = 0; jb < VB; ++jb) {
        floatx4 xc[TPW], xb[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          xc[t] = *reinterpret_cast<const floatx4*>(vc[t] + 16 * jb + 4 * g4);
          xb[t] = *reinterpret_cast<const floatx4*>(vb[t] + 16 * jb + 4 * g4);
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const floatx4 w = bq[64 * (3 * jb + mu)];
          const float wv[4] = {w.x, w.y, w.z, w.w};
          floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
          if (TAIL > 0) z = tq[16 * (3 * jb + mu)];
          const float zv[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            float av[TPW];
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
              const float xcs = s == 0 ? xc[t].x : s == 1 ? xc[t].y : s == 2 ? xc[t].z : xc[t].w;
              const float xbs = s == 0 ? xb[t].x : s == 1 ? xb[t].y : s == 2 ? xb[t].z : xb[t].w;
              av[t] = pc[t][mu] * xcs + qc[t][mu] * xbs;
            }
            // the 16x16x4 products of all tiles first, then the short tail products
#pragma unroll
            for (int t = 0; t < TPW; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], wv[s], acc[t], 0, 0, 0);
            if (TAIL > 0 && nt == 0)
#pragma unroll
              for (int t = 0; t < TPW; ++t) tacc[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[t], zv[s], tacc[t], 0, 0, 0);
          }
        }
      }
      // the next tile's fields and geometry are requested between the volume and face steps
      prefetch(nxt);
#pragma unroll
      for (int fb = 0; fb < QF; ++fb) {
        // the exterior traces of the next tile are issued in two halves among the last MFMAs
        // of the contraction, so that the scattered loads overlap matrix work; staging and
        // write-out then cover their latency
        if (fb == QF / 2) gather(nxt, fcb[more ? par ^ 1 : par], 0, FIT / 2);
        floatx4 xf[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) xf[t] = *reinterpret_cast<const floatx4*>(fl[t] + 16 * fb);
        const floatx4 w = bq[64 * (QV + fb)];
        const float wv[4] = {w.x, w.y, w.z, w.w};
        floatx4 z = floatx4{0.f, 0.f, 0.f, 0.f};
        if (TAIL > 0) z = tq[16 * (QV + fb)];
        const float zv[4] = {z.x, z.y, z.z, z.w};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float xs[TPW];
#pragma unroll
          for (int t = 0; t < TPW; ++t) xs[t] = s == 0 ? xf[t].x : s == 1 ? xf[t].y : s == 2 ? xf[t].z : xf[t].w;
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs[t], wv[s], acc[t], 0, 0, 0);
          if (TAIL > 0 && nt == 0)
#pragma unroll
            for (int t = 0; t < TPW; ++t) tacc[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(xs[t], zv[s], tacc[t], 0, 0, 0);
        }
      }
      gather(nxt, fcb[more ? par ^ 1 : par], FIT / 2, FIT);
#pragma unroll
      for (int r = 0; r < VR; ++r) {
        float xc1[TPW], xb1[TPW];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
          xc1[t] = vc[t][16 * VB + 4 * r + g4];   // columns >= Np read the zero padding
          xb1[t] = vb[t][16 * VB + 4 * r + g4];
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const float w = bs[64 * (3 * r + mu)];
          const float zs = TAIL > 0 ? ts[16 * (3 * r + mu)] : 0.f;
          float av[TPW];
#pragma unroll
          for (int t = 0; t < TPW; ++t) av[t] = pc[t][mu] * xc1[t] + qc[t][mu] * xb1[t];
#pragma unroll
          for (int t = 0; t < TPW; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], w, acc[t], 0, 0, 0);
          if (TAIL > 0 && nt == 0)
#pragma unroll
            for (int t = 0; t < TPW; ++t) tacc[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[t], zs, tacc[t], 0, 0, 0);
        }
      }
    }

    if (D::PRIO) __builtin_amdgcn_s_setprio(0);
    // tail: sum the partial results of the four k-groups (lanes li, li + 16, li + 32, li + 48)
    if (TAIL > 0 && nt == 0) {
#pragma unroll
      for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float v = tacc[t][i];
          v += __shfl_xor(v, 16);
          v += __shfl_xor(v, 32);
          tacc[t][i] = v;
        }
    }
    __syncthreads();   // flux rows are read: reuse them for the staging

    // ---- stage the right-hand side [e][f][n] in LDS. 16x16x4 result: lane (li, g4), register
    // i = row 4 g4 + i, node 16 nt + li. Tail (column tile 0 waves, lanes g4 = 0): lane li,
    // register i = row 4 (li / 4) + i, node 16 NT + li mod 4.
    float* stage = gl;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = wave + 4 * t;
      if (tt < TILES) {
        const int f = tt / NT;
#pragma unroll
        for (int i = 0; i < 4; ++i) stage[(4 * g4 + i) * ES + f * NPP + 16 * nt + li] = acc[t][i];
        if (TAIL > 0 && nt == 0 && g4 == 0 && (li & 3) < TAIL) {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            stage[(4 * (li >> 2) + i) * ES + f * NPP + 16 * NT + (li & 3)] = tacc[t][i];
        }
      }
    }
    __syncthreads();

    // ---- update and write out, coalesced. Buffer stores bounded by the tile's words, issued by
    // every lane: a chunk past the tile (the partial last round, a ragged tile) is dropped by the
    // range check, so no store sits on a conditional path (the compiler's wait counting would
    // then make the next flux phase wait for these stores to complete).
    {
      const int nbytes = nel * 6 * NPP * 4;
      const __amdgpu_buffer_rsrc_t ro = tile_rsrc(out + tb, nbytes);
      const __amdgpu_buffer_rsrc_t rr = tile_rsrc(res + tb, nbytes);
      int tw = tid;   // opaque, like tz
      asm volatile("" : "+v"(tw));
#pragma unroll
      for (int j = 0; j < CPC; ++j) {
        const int c = tw + j * kThreads;
        const int o = slot(4 * min(c, TC - 1));
        const floatx4 h = *reinterpret_cast<const floatx4*>(stage + o);
        if (STAGE) {
          const floatx4 u = *reinterpret_cast<const floatx4*>(up_s + o);
          const floatx4 rv = pad_zero(c, floatx4{ca * rs[j].x + cdt * h.x, ca * rs[j].y + cdt * h.y,
                                                 ca * rs[j].z + cdt * h.z, ca * rs[j].w + cdt * h.w});
          const floatx4 un = floatx4{u.x + cb * rv.x, u.y + cb * rv.y, u.z + cb * rv.z, u.w + cb * rv.w};
          // residual and state are touched once per stage: nontemporal, they leave L2 to the
          // neighbour traces
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, rv), rr, c * 16, 0, kNonTemporal);
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, un), ro, c * 16, 0, kNonTemporal);
        } else {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, pad_zero(c, h)), ro, c * 16, 0, 0);
        }
      }
    }
    // face records of the tile after next replace those of this tile
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();   // the next tile overwrites up_s, gt, fcb and gl
  }
}

// ---------------------------------------------------------------------------------------
// MFMA form of the fused stage for the higher orders (FP32, N = 5, 6).
//
// The same contraction as above (contravariant fluxes; rhs = OpCat x [G; Fscale/2 flux]; the
// k-steps in volume quads, face quads and volume singles, each lane reading four k-steps with
// one 16-byte LDS read) with the sizes of the higher orders in mind: the operator is too large
// to copy into LDS per workgroup (NT x KS x 256 B = 67 KB at N = 5), so each wave owns one
// 16-node column tile and keeps that tile's operator fragments in VGPRs for the life of the
// persistent workgroup (KS = 66 / 91 per lane). A tile holds 8 elements (48 rows = 3 row
// tiles, all handled by every wave); the last column tile is zero-padded (operator rows >= Np
// are zero), which replaces the 4x4x1 tail.
template <int N>
struct HDims {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, Nf4 = Dims<N>::Nf4;
  static constexpr int E = 8;                         // elements per tile
  static constexpr int ROWS = 6 * E;                  // (field, element) rows, field-major
  static constexpr int RT = ROWS / 16;                // row tiles, all owned by every wave
  static constexpr int NT = (Np + 15) / 16;           // column tiles (last one padded)
  static constexpr int THREADS = 64 * NT;             // one wave per column tile
  static constexpr int TW = E * 6 * Np;
  static constexpr int TW4 = TW / 4;
  static constexpr int CPT = (TW4 + THREADS - 1) / THREADS;
  static constexpr int NPP = (Np + 3) / 4 * 4;
  static constexpr int ES = 6 * NPP + 4;              // = 4 mod 8 (conflict-free rows)
  static constexpr int NF = (Nf4 + 15) / 16 * 16;
  static constexpr int RSL = NF + 4;
  static constexpr int KV = 3 * NPP;
  static constexpr int KD = KV + NF;
  static constexpr int KS = KD / 4;
  static constexpr int VB = NPP / 16;
  static constexpr int VR = (NPP - 16 * VB) / 4;
  static constexpr int QV = 3 * VB, QF = NF / 16;
  static constexpr int NQ = QV + QF;
  static constexpr int FIT = (E * Nf4 + THREADS - 1) / THREADS;
  static constexpr int OPC = NT * KS * 64;            // fragment-ordered operator, no tail
  // exterior traces gathered one tile ahead (registers live across the contraction) where the
  // register file allows two waves per SIMD; otherwise at the start of the flux phase
  static constexpr bool AHEAD = N == 5;
  // N = 7: the operator strip (126 VGPRs per lane) is streamed from L2 per tile instead of kept
  // resident, as in the FP64 kernel of these orders (1809 against 1951 us per stage at K =
  // 196,608; at N = 5, 6 the resident strip is faster: 464 / 1214 against 503 / 1388 us)
  static constexpr bool STREAM = N == 7;
  static constexpr int LA = STREAM ? 3 : 1;           // streamed quads in flight
  static_assert(4 * NQ + 3 * VR == KS, "k-steps are quads and singles");
  static_assert(TW % 4 == 0, "a tile is a whole number of float4 chunks");
  static_assert(NPP == Np, "rows need no padding: 16-byte chunks of a tile map to the LDS rows");
  static_assert(TW <= ROWS * RSL, "staging must fit in the flux rows");
  static_assert(ROWS % 16 == 0, "whole row tiles");
};

template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(HDims<N>::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void hmfma_stage_kernel(
    const float* __restrict__ u_in, float* __restrict__ out, float* __restrict__ res,
    const float* __restrict__ geo, const int32_t* __restrict__ fcode, const float* __restrict__ mat,
    const float* __restrict__ opf, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, float ca, float cb, float cdt, SrcArgs inc) {
  using D = HDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES,
                NF = D::NF, KS = D::KS, RSL = D::RSL, RT = D::RT, FIT = D::FIT,
                TW4 = D::TW4, CPT = D::CPT, VB = D::VB, VR = D::VR, QV = D::QV, QF = D::QF,
                NQ = D::NQ, NTH = D::THREADS;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;
  constexpr int GPT = (GW + NTH - 1) / NTH;
  __shared__ __align__(16) float up_s[E * ES];        // field tile [e][f][n], element stride ES
  __shared__ __align__(16) float gl[D::ROWS * RSL];   // flux rows [f E + e][fj]; later staging
  __shared__ float gt[GW];
  __shared__ __align__(16) float wmat[MAT ? E * 4 * dgh::kMatFace : 4];   // MAT: face weights [e][f][A B C D]
  __shared__ int32_t fcb[2][E * 4];                   // face records: this tile, the next
  __shared__ uint8_t nbr_s[96 * NFP];
  __shared__ uint8_t fm_s[4 * NFP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int nt = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's column tile
  const int g4 = lane >> 4, li = lane & 15;
  // slot in up_s of word q of a tile of the [K][6][Np] field arrays
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NP);
    return e * ES + (q - e * 6 * NP);
  };

  const int nwg = gridDim.x / kXcds;
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  // once per workgroup: this wave's operator fragments (registers, unless streamed) and the
  // node tables
  floatx4 bq[D::STREAM ? 1 : NQ];
  float bs[3 * VR > 0 ? 3 * VR : 1];
  if constexpr (!D::STREAM) {
    const floatx4* src = reinterpret_cast<const floatx4*>(opf + size_t(nt) * KS * 64) + lane;
#pragma unroll
    for (int q = 0; q < NQ; ++q) bq[q] = src[64 * q];
    const float* s1 = opf + size_t(nt) * KS * 64 + NQ * 256 + lane;
#pragma unroll
    for (int q = 0; q < 3 * VR; ++q) bs[q] = s1[64 * q];
  }
  for (int q = tid; q < 96 * NFP; q += NTH) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += NTH) fm_s[q] = uint8_t(fmask[q]);

  // prefetch registers, as in the kernel above: fields and geometry of the next tile, the
  // exterior traces of its face nodes, the face records of the tile after it
  int tq = tid;
  asm volatile("" : "+v"(tq));
  floatx4 pu[CPT];
  float pg[GPT];
  float nup[FIT][6];
  int32_t pf = 0;
  float pm = 0.f, pw = 0.f;
  const size_t fc_last = size_t(K) * 4 - 1;
  // every load issued on every path, indices clamped into the arrays (as in the kernel above)
  const size_t chunk_last = size_t(K) * 6 * NP / 4 - 1;
  const floatx4* u4 = reinterpret_cast<const floatx4*>(u_in);
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) pu[r] = u4[min(size_t(t) * TW4 + min(tid + r * NTH, TW4 - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * NTH, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);   // word qw % 16 of the face weights of element qw / 16
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  auto gather = [&](int t, const int32_t* fcv) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = min(tq + r * NTH, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const float* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NP + nn : size_t(e0 + e) * 6 * NP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NP];
    }
  };
  int par = 0;
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  if (D::AHEAD) gather(tile, fcb[0]);
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    const size_t tb = size_t(base) * 6 * NP;
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;

    if (full) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int q = tid + r * NTH;
        if (q < TW4) *reinterpret_cast<floatx4*>(up_s + slot(4 * q)) = pu[r];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) up_s[slot(q)] = u_in[tb + q];
      if (MAT) {
        for (int q = tid; q < 2 * nel; q += NTH)
          up_s[(q >> 1) * ES + 6 * NPP + (q & 1)] = mat[(size_t(base) + (q >> 1)) * dgh::kMatStride + (q & 1)];
        for (int q = tid; q < 16 * nel; q += NTH)
          wmat[q] = mat[(size_t(base) + q / 16) * dgh::kMatStride + dgh::kMatFace + (q & 15)];
      }
      for (int q = tid; q < nel * G; q += NTH) gt[q] = geo[size_t(base) * G + q];
    }
    __syncthreads();

    floatx4 rs4[CPT];

    __builtin_amdgcn_s_setprio(2);   // issue priorities as in the kernel above
    // ---- face fluxes (as in the kernel above)
    const int32_t* fc = fcb[par];
    if (!D::AHEAD) gather(tile, fc);
    {
      floatx4 wm[FIT];
      if (MAT) {
#pragma unroll
        for (int r = 0; r < FIT; ++r) {
          const int q = min(tq + r * NTH, nel * NF4 - 1);
          const int e = q / NF4, f = (q - e * NF4) / NFP;
          wm[r] = *reinterpret_cast<const floatx4*>(wmat + 16 * e + 4 * f);
        }
      }
      if constexpr (NF > NF4)
        for (int q = tid; q < D::ROWS * (NF - NF4); q += NTH) {
          const int row = q / (NF - NF4);
          gl[row * RSL + NF4 + (q - row * (NF - NF4))] = 0.f;
        }
#pragma unroll
      for (int r = 0; r < FIT; ++r) {
        const int q = tq + r * NTH;
        if (q < nel * NF4) {
          const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
          const float* g = gt + e * G + dgh::kGeoNormal + 4 * f;
          const float nx = g[0], ny = g[1], nz = g[2], hs = 0.5f * g[3];
          const float* um = up_s + e * ES + fm_s[f * NFP + j];
          float m[6], d[6];
#pragma unroll
          for (int c = 0; c < 6; ++c) m[c] = um[c * NP];
          const int code = fc[e * 4 + f];
          if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
          face_jump(code, m, nup[r], d);
          const float w[4] = {wm[r].x, wm[r].y, wm[r].z, wm[r].w};
          upwind_flux(MAT, nx, ny, nz, hs, w, d, gl + e * RSL + fj, E * RSL);
        }
      }
    }
    __syncthreads();
    // streamed operator: the first quads and the singles of this wave's strip, issued before
    // the next tile's prefetch; the base address passes through an empty asm so the loads stay
    // in the tile loop
    constexpr int LA = D::LA;
    floatx4 wb[LA];
    if constexpr (D::STREAM) {
      const float* opw = opf + size_t(nt) * KS * 64;
      asm volatile("" : "+s"(opw));
      const floatx4* bqs = reinterpret_cast<const floatx4*>(opw) + lane;
#pragma unroll
      for (int i = 0; i < LA; ++i) wb[i] = bqs[64 * i];
#pragma unroll
      for (int i = 0; i < 3 * VR; ++i) bs[i] = opw[NQ * 256 + 64 * i + lane];
    }
    // operator quad q: resident, or the one loaded LA quads ago (its buffer takes quad q + LA)
    auto quad = [&](int q) __attribute__((always_inline)) {
      if constexpr (D::STREAM) {
        const floatx4 w = wb[q % LA];
        if (q + LA < NQ) {
          const float* opw = opf + size_t(nt) * KS * 64;
          asm volatile("" : "+s"(opw));
          wb[q % LA] = reinterpret_cast<const floatx4*>(opw)[64 * (q + LA) + lane];
        }
        return w;
      } else {
        return bq[q];
      }
    };
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r)
        rs4[r] = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(res) +
                                            min(size_t(tile) * TW4 + min(tid + r * NTH, TW4 - 1), chunk_last));
    }
    prefetch(nxt);

    __builtin_amdgcn_s_setprio(3);
    // ---- contraction: this wave's column tile against the three row tiles. Row tile t holds
    // rows 16 t + li, row = f E + e (two fields of 8 elements).
    floatx4 acc[RT];
    {
      float pc[RT][3], qc[RT][3];
      const float* vc[RT];
      const float* vb[RT];
      const float* fl[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int row = 16 * t + li;
        const int f = row / E, e = row - f * E;
        const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
        const int srcf = f < 3 ? 3 : 0;
        const float sg = f < 3 ? 1.f : -1.f;
        const float* cm = gt + e * G;
        const float sm = MAT ? sg * up_s[e * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          pc[t][mu] = sm * cm[3 * mu + b];
          qc[t][mu] = -sm * cm[3 * mu + c];
        }
        vc[t] = up_s + e * ES + (srcf + c) * NPP;
        vb[t] = up_s + e * ES + (srcf + b) * NPP;
        fl[t] = gl + row * RSL + 4 * g4;
      }
#pragma unroll
      for (int jb = 0; jb < VB; ++jb) {
        floatx4 xc[RT], xb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          xc[t] = *reinterpret_cast<const floatx4*>(vc[t] + 16 * jb + 4 * g4);
          xb[t] = *reinterpret_cast<const floatx4*>(vb[t] + 16 * jb + 4 * g4);
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const floatx4 w = quad(3 * jb + mu);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            const float ws = s == 0 ? w.x : s == 1 ? w.y : s == 2 ? w.z : w.w;
            float av[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t) {
              const float xcs = s == 0 ? xc[t].x : s == 1 ? xc[t].y : s == 2 ? xc[t].z : xc[t].w;
              const float xbs = s == 0 ? xb[t].x : s == 1 ? xb[t].y : s == 2 ? xb[t].z : xb[t].w;
              av[t] = pc[t][mu] * xcs + qc[t][mu] * xbs;
            }
#pragma unroll
            for (int t = 0; t < RT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[t], ws, acc[t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int fb = 0; fb < QF; ++fb) {
        floatx4 xf[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) xf[t] = *reinterpret_cast<const floatx4*>(fl[t] + 16 * fb);
        const floatx4 w = quad(QV + fb);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const float ws = s == 0 ? w.x : s == 1 ? w.y : s == 2 ? w.z : w.w;
#pragma unroll
          for (int t = 0; t < RT; ++t) {
            const float xs = s == 0 ? xf[t].x : s == 1 ? xf[t].y : s == 2 ? xf[t].z : xf[t].w;
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs, ws, acc[t], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int r = 0; r < VR; ++r) {
        float xc1[RT], xb1[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          xc1[t] = vc[t][16 * VB + 4 * r + g4];   // columns >= Np read the zero padding
          xb1[t] = vb[t][16 * VB + 4 * r + g4];
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const float w = bs[3 * r + mu];
#pragma unroll
          for (int t = 0; t < RT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(pc[t][mu] * xc1[t] + qc[t][mu] * xb1[t], w, acc[t], 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    if (D::AHEAD) gather(nxt, fcb[more ? par ^ 1 : par]);
    __syncthreads();   // flux rows are read: reuse them for the staging

    // ---- stage the right-hand side [e][f][n]: lane (li, g4), register i = row 16 t + 4 g4 + i,
    // node 16 nt + li (nodes >= Np are the padding of the last column tile)
    float* stage = gl;
    const int col = 16 * nt + li;
    if (col < NP) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * t + 4 * g4 + i;
          const int f = row / E, e = row - f * E;
          stage[(e * 6 + f) * NP + col] = acc[t][i];
        }
    }
    __syncthreads();

    // ---- update and write out, coalesced
    if (full) {
      floatx4* o4 = reinterpret_cast<floatx4*>(out + tb);
      floatx4* r4 = reinterpret_cast<floatx4*>(res + tb);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int q = tid + r * NTH;
        if (q < TW4) {
          const floatx4 h = reinterpret_cast<const floatx4*>(stage)[q];
          if (STAGE) {
            const floatx4 u = *reinterpret_cast<const floatx4*>(up_s + slot(4 * q));
            const floatx4 rv = ca * rs4[r] + cdt * h;
            __builtin_nontemporal_store(rv, r4 + q);
            __builtin_nontemporal_store(u + cb * rv, o4 + q);
          } else {
            o4[q] = h;
          }
        }
      }
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) {
        const float h = stage[q];
        if (STAGE) {
          const float rv = ca * res[tb + q] + cdt * h;
          res[tb + q] = rv;
          out[tb + q] = up_s[slot(q)] + cb * rv;
        } else {
          out[tb + q] = h;
        }
      }
    }
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();   // the next tile overwrites up_s, gt, fcb and gl
  }
}

// ---------------------------------------------------------------------------------------
// MFMA form of the fused stage in FP64 (N = 3).
//
// The same contraction as the FP32 kernels (contravariant fluxes; rhs = OpCat x [G; Fscale/2
// flux]; k-steps in volume quads, face quads and volume singles; the operator table in the
// same fragment order), on v_mfma_f64_16x16x4f64. On gfx950 the FP64 matrix rate equals the
// FP64 vector rate (64 cycles per 16x16x4 step), so the point of the matrix path is that
// the multiply-adds leave the VALU free for the operand, the fluxes and the memory phases.
// The Np mod 16 tail columns run on v_mfma_f64_4x4x4f64, whose A operand has the lane layout
// of the 16x16x4 one (lane 16 k + 4 b + r holds row 4 b + r of k-step k): it takes the same
// operand register, and its B operand (lane 16 k + 4 b + c) is the tail operator replicated
// over the four row blocks b, which is the (k-group, column) order of the FP32 tail table.
// Result layouts: 16x16x4, lane (li, g4) register i = row g4 + 4 i, column li; 4x4x4, lane
// (li, g4) = row 4 (li / 4) + g4, column li mod 4.
//
// One wave per 16-row tile: a tile of 8 elements has 48 (field, element) rows, field-major,
// and wave t computes all column tiles and the tail of rows 16 t .. 16 t + 15, so the three
// waves carry equal matrix work. Fields, fluxes and the operator table sit in LDS (47 KB: three
// workgroups per CU; 16-element tiles with six waves and two workgroups per CU ran 16 %
// slower); the next tile's fields, geometry and exterior traces are loaded into registers
// during this tile, every load issued on every path with clamped indices (as in the FP32
// kernels). Issue priorities as in the FP32 kernels (contraction 3, fluxes 2, memory phases 0).
// The residual is read and the new state and residual written with nontemporal hints: each is
// touched once per stage, so they need not displace the neighbour traces in L2.
template <int N>
struct DDims {
  using M = MDims<N>;                                 // operand and operator geometry
  static constexpr int Np = M::Np, Nfp = M::Nfp, Nf4 = M::Nf4;
  static constexpr int E = 8;                         // elements per tile
  static constexpr int WAVES = 6 * E / 16, THREADS = 64 * WAVES;   // one wave per 16-row tile
  static constexpr int NPP = M::NPP;                  // row stride of the field arrays
  static constexpr int ES = 6 * NPP + 2;              // element stride in LDS (doubles, = 2 mod 4)
  static constexpr int NF = M::NF, RSL = NF + 2;      // flux row stride (doubles, = 2 mod 4)
  static constexpr int KS = M::KS, VB = M::VB, VR = M::VR, QV = M::QV, QF = M::QF, NQ = M::NQ;
  static constexpr int NT = M::NT, TAIL = M::TAIL;
  static constexpr int TW = E * 6 * NPP;              // doubles per tile
  static constexpr int TC = TW / 2;                   // 16-byte chunks per tile
  static constexpr int CPT = (TC + THREADS - 1) / THREADS;
  static constexpr int FIT = (E * Nf4 + THREADS - 1) / THREADS;
  static constexpr int OPC = M::OPC;
  static_assert(NPP == Np, "FP64 rows are unpadded");
  static_assert((6 * NPP) % 2 == 0, "16-byte chunks do not straddle elements");
  static_assert(TAIL > 0 && TAIL <= 4, "one 4x4x4 tail block");
  static_assert(E * ES <= 6 * E * RSL, "staging fits in the flux rows");
};

typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(DDims<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3, 3))) void dmfma_stage_kernel(
    const double* __restrict__ u_in, double* __restrict__ out, double* __restrict__ res,
    const double* __restrict__ geo, const int32_t* __restrict__ fcode, const double* __restrict__ mat,
    const double* __restrict__ opf, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, double ca, double cb, double cdt, SrcArgs inc) {
  using D = DDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES, NF = D::NF,
                KS = D::KS, RSL = D::RSL, NT = D::NT, TAIL = D::TAIL, FIT = D::FIT, TC = D::TC, CPT = D::CPT,
                VB = D::VB, VR = D::VR, QV = D::QV, QF = D::QF, NQ = D::NQ, NTH = D::THREADS;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;
  constexpr int GPT = (GW + NTH - 1) / NTH;
  __shared__ __align__(16) double up_s[E * ES];            // field tile [e][f][n]
  __shared__ __align__(16) double gl[6 * E * RSL];         // flux rows [f E + e][fj]; later staging
  __shared__ __align__(16) double bfs[NT * KS * 64];       // operator fragments
  __shared__ __align__(16) double tops[KS * 16];           // tail operator (k-group, column)
  __shared__ double gt[GW];
  __shared__ __align__(16) double wmat[MAT ? E * 4 * dgh::kMatFace : 2];   // MAT: [e][f][A B C D]
  __shared__ int32_t fcb[2][E * 4];
  __shared__ uint8_t nbr_s[96 * NFP];
  __shared__ uint8_t fm_s[4 * NFP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int fw = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's 16-row tile
  const int g4 = lane >> 4, li = lane & 15;
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NPP);
    return e * ES + (q - e * 6 * NPP);
  };

  const int nwg = gridDim.x / kXcds;
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  for (int q = tid; q < NT * KS * 64; q += NTH) bfs[q] = opf[q];
  for (int q = tid; q < KS * 16; q += NTH) tops[q] = opf[NT * KS * 64 + q];
  for (int q = tid; q < 96 * NFP; q += NTH) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += NTH) fm_s[q] = uint8_t(fmask[q]);
  for (int q = tid; q < E * ES; q += NTH) up_s[q] = 0.0;
  __syncthreads();

  int tq = tid;
  if (MAT) asm volatile("" : "+v"(tq));
  doublex2 pu[CPT];
  double pg[GPT];
  double nup[FIT][6];
  int32_t pf = 0;
  double pm = 0.0, pw = 0.0;
  const size_t fc_last = size_t(K) * 4 - 1;
  const size_t chunk_last = size_t(K) * 6 * NPP / 2 - 1;
  const doublex2* u2 = reinterpret_cast<const doublex2*>(u_in);
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) pu[r] = u2[min(size_t(t) * TC + min(tid + r * NTH, TC - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * NTH, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  auto gather = [&](int t, const int32_t* fcv) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = min(tq + r * NTH, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const double* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NPP + nn : size_t(e0 + e) * 6 * NPP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NPP];
    }
  };
  int par = 0;
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  gather(tile, fcb[0]);
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  // the first tile's loads complete here, once per workgroup, so that the waits inside the loop
  // are counted from the loop's own order of issue
  __builtin_amdgcn_s_waitcnt(0);

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    const size_t tb = size_t(base) * 6 * NPP;
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;

    // ---- tile into LDS
    if (full) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if ((r + 1) * NTH <= TC || c < TC) *reinterpret_cast<doublex2*>(up_s + slot(2 * c)) = pu[r];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      // a ragged tile comes from the prefetch registers too: the clamped loads read the right
      // words below the end of the arrays (no load on this path)
      const int nc = nel * 6 * NPP / 2;
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if (c < nc) *reinterpret_cast<doublex2*>(up_s + slot(2 * c)) = pu[r];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < nel * G) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * nel) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * nel) wmat[tid] = pw;
    }
    __syncthreads();

    // ---- face fluxes from the exterior traces gathered during the previous tile
    const int32_t* fc = fcb[par];
    __builtin_amdgcn_s_setprio(2);
    {
      if constexpr (NF > NF4)
        for (int q = tid; q < 6 * E * (NF - NF4); q += NTH) {
          const int row = q / (NF - NF4);
          gl[row * RSL + NF4 + (q - row * (NF - NF4))] = 0.0;
        }
#pragma unroll
      for (int r = 0; r < FIT; ++r) {
        const int q = tq + r * NTH;
        if (q < nel * NF4) {
          const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
          const double* g = gt + e * G + dgh::kGeoNormal + 4 * f;
          const double nx = g[0], ny = g[1], nz = g[2], hs = 0.5 * g[3];
          const double* um = up_s + e * ES + fm_s[f * NFP + j];
          double m[6], d[6], w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int c = 0; c < 6; ++c) m[c] = um[c * NPP];
          const int code = fc[e * 4 + f];
          if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
          face_jump(code, m, nup[r], d);
          if (MAT) {
            const doublex2 w01 = *reinterpret_cast<const doublex2*>(wmat + 16 * e + 4 * f);
            const doublex2 w23 = *reinterpret_cast<const doublex2*>(wmat + 16 * e + 4 * f + 2);
            w[0] = w01.x, w[1] = w01.y, w[2] = w23.x, w[3] = w23.y;
          }
          upwind_flux(MAT, nx, ny, nz, hs, w, d, gl + e * RSL + fj, E * RSL);
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    doublex2 rs[CPT];
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r)
        rs[r] = __builtin_nontemporal_load(reinterpret_cast<const doublex2*>(res) +
                                           min(size_t(tile) * TC + min(tid + r * NTH, TC - 1), chunk_last));
    }
    // the next tile's fields and geometry, then its exterior traces
    prefetch(nxt);
    gather(nxt, fcb[more ? par ^ 1 : par]);

    // ---- contraction of row tile fw: row 16 fw + li = (field f, element el)
    __builtin_amdgcn_s_setprio(3);
    doublex4 acc[NT];
    double tacc = 0.0;
    {
      const int row = 16 * fw + li, f = row / E, el = row - f * E;
      const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
      const int srcf = f < 3 ? 3 : 0;            // H feeds the E rows, E the H rows
      const double sg = f < 3 ? 1.0 : -1.0;
      const double* cm = gt + el * G;
      const double sm = MAT ? sg * up_s[el * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
      double pc[3], qc[3];   // operand = pc[mu] V_c + qc[mu] V_b
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        pc[mu] = sm * cm[3 * mu + b];
        qc[mu] = -sm * cm[3 * mu + c];
      }
      const double* vc = up_s + el * ES + (srcf + c) * NPP;
      const double* vb = up_s + el * ES + (srcf + b) * NPP;
      const double* fl = gl + row * RSL + 4 * g4;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
      auto ld4 = [](const double* p) __attribute__((always_inline)) {
        const doublex2 lo = *reinterpret_cast<const doublex2*>(p);
        const doublex2 hi = *reinterpret_cast<const doublex2*>(p + 2);
        return doublex4{lo.x, lo.y, hi.x, hi.y};
      };
      const double* bq = bfs + 4 * lane;                  // quad q of column tile t: bq + (t KS + 4 q) 64
      const double* bs = bfs + NQ * 256 + lane;           // single s of column tile t: bs + t KS 64 + 64 s
      const int tl = 4 * g4 + (li & 3);
      const double* tq4 = tops + 4 * tl;                  // tail quad q: tq4 + 64 q
      const double* ts1 = tops + NQ * 64 + tl;            // tail single s: ts1 + 16 s
      auto step = [&](double av, const doublex4 (&w)[NT], const doublex4& z, int s) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, w[t][s], acc[t], 0, 0, 0);
        tacc = __builtin_amdgcn_mfma_f64_4x4x4f64(av, z[s], tacc, 0, 0, 0);
      };
#pragma unroll
      for (int jb = 0; jb < VB; ++jb) {
        const doublex4 xc = ld4(vc + 16 * jb + 4 * g4);
        const doublex4 xb = ld4(vb + 16 * jb + 4 * g4);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const int q = 3 * jb + mu;
          doublex4 w[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) w[t] = ld4(bq + (t * KS * 64) + 256 * q);
          const doublex4 z = ld4(tq4 + 64 * q);
#pragma unroll
          for (int s = 0; s < 4; ++s) step(pc[mu] * xc[s] + qc[mu] * xb[s], w, z, s);
        }
      }
#pragma unroll
      for (int fb = 0; fb < QF; ++fb) {
        const int q = QV + fb;
        const doublex4 xf = ld4(fl + 16 * fb);
        doublex4 w[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t] = ld4(bq + (t * KS * 64) + 256 * q);
        const doublex4 z = ld4(tq4 + 64 * q);
#pragma unroll
        for (int s = 0; s < 4; ++s) step(xf[s], w, z, s);
      }
#pragma unroll
      for (int r = 0; r < VR; ++r) {
        const double xc1 = vc[16 * VB + 4 * r + g4];   // columns >= Np read the zero padding
        const double xb1 = vb[16 * VB + 4 * r + g4];
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const int sgl = 3 * r + mu;
          const double av = pc[mu] * xc1 + qc[mu] * xb1;
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bs[t * KS * 64 + 64 * sgl], acc[t], 0, 0, 0);
          tacc = __builtin_amdgcn_mfma_f64_4x4x4f64(av, ts1[16 * sgl], tacc, 0, 0, 0);
        }
      }
    }
    __syncthreads();   // flux rows are read: reuse them for the staging

    // ---- stage the right-hand side [e][f][n] (laid out like up_s)
    __builtin_amdgcn_s_setprio(0);
    double* stage = gl;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * fw + g4 + 4 * i, f = row / E, el = row - f * E;
        stage[el * ES + f * NPP + 16 * t + li] = acc[t][i];
      }
    if ((li & 3) < TAIL) {
      const int row = 16 * fw + 4 * (li >> 2) + g4, f = row / E, el = row - f * E;
      stage[el * ES + f * NPP + 16 * NT + (li & 3)] = tacc;
    }
    __syncthreads();

    // ---- update and write out, 16-byte chunks: buffer stores bounded by the tile's words, issued
    // by every lane (a chunk past the tile is dropped by the range check; no store on a
    // conditional path, so the next flux phase does not wait for these stores)
    {
      const int nbytes = nel * 6 * NPP * 8;
      const __amdgpu_buffer_rsrc_t ro = tile_rsrc(out + tb, nbytes);
      const __amdgpu_buffer_rsrc_t rr = tile_rsrc(res + tb, nbytes);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        const int o = slot(2 * min(c, TC - 1));
        const doublex2 h = *reinterpret_cast<const doublex2*>(stage + o);
        if (STAGE) {
          const doublex2 u = *reinterpret_cast<const doublex2*>(up_s + o);
          const doublex2 rv = doublex2{ca * rs[r].x + cdt * h.x, ca * rs[r].y + cdt * h.y};
          const doublex2 un = doublex2{u.x + cb * rv.x, u.y + cb * rv.y};
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, rv), rr, c * 16, 0, kNonTemporal);
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, un), ro, c * 16, 0, kNonTemporal);
        } else {
          __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(uint4v, h), ro, c * 16, 0, 0);
        }
      }
    }
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();   // the next tile overwrites up_s, gt, fcb and gl
  }
}

// ---------------------------------------------------------------------------------------
// MFMA form of the fused stage in FP64 at N = 4..7.
//
// The contraction of the FP32 kernel for these orders (8-element tiles, three 16-row tiles
// owned by every wave, one wave per 16-node column tile, the last one padded; the operator
// table in the same fragment order, in FP64) on v_mfma_f64_16x16x4f64. In FP64 a wave's
// operator strip is 2 KD VGPRs per lane (264 at N = 7), too large to keep resident, and the
// whole operator (100-480 KB) does not fit in LDS beside the tile, so each wave streams its
// strip from L2 (the table is a few hundred KB and every workgroup of an XCD reads it) with
// LA quads in flight; each operator value a lane loads (8 bytes) feeds RT matrix steps of 16
// multiply-adds per lane, i.e. 1/6 byte of L2 reads per lane and multiply-add. The first quads
// are issued before the next tile's prefetch, so their waits do not include those HBM loads.
// Exterior traces of the next tile are gathered after the contraction (their registers are not
// live across it); the residual is loaded after them, for the update. Issue priorities and
// nontemporal residual and state I/O as in the other contraction kernels. Result layout: lane
// (li, g4) register i = row 16 t + g4 + 4 i of row tile t, node 16 nt + li. At N = 4 (35
// nodes) the LDS rows are padded to 36 words (the pad word stays zero, so the last volume
// single reads zero there); the HBM rows stay unpadded, so a 16-byte chunk of the tile may
// straddle two LDS rows and is moved as two words.
template <int N>
struct WDims {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, Nf4 = Dims<N>::Nf4;
  static constexpr int E = 8;                         // elements per tile
  static constexpr int ROWS = 6 * E, RT = ROWS / 16;  // (field, element) rows, field-major
  static constexpr int NPP = (Np + 3) / 4 * 4;        // LDS row of a field (N = 4: one zero pad word)
  static constexpr int NT = (NPP + 15) / 16;          // column tiles (last one padded)
  static constexpr int THREADS = 64 * NT;             // one wave per column tile
  static constexpr int NF = (Nf4 + 15) / 16 * 16;
  static constexpr int KV = 3 * NPP, KD = KV + NF, KS = KD / 4;
  static constexpr int VB = NPP / 16, VR = (NPP - 16 * VB) / 4;
  static constexpr int QV = 3 * VB, QF = NF / 16, NQ = QV + QF;
  static constexpr int FIT = (E * Nf4 + THREADS - 1) / THREADS;
  static constexpr int OPC = NT * KS * 64;            // fragment-ordered operator, no tail
  static constexpr int ES = 6 * NPP + 2;              // element stride in LDS (doubles, = 2 mod 4)
  static constexpr int RSL = NF + 2;                  // flux row stride (doubles, = 2 mod 4)
  static constexpr int TW = E * 6 * Np;               // doubles per tile (HBM rows are unpadded)
  static constexpr int TC = TW / 2;                   // 16-byte chunks per tile
  static constexpr int CPT = (TC + THREADS - 1) / THREADS;
  static constexpr int LA = 3;                        // operator quads in flight per wave
  static_assert(4 * NQ + 3 * VR == KS, "k-steps are quads and singles");
  static_assert((6 * Np) % 2 == 0, "16-byte chunks do not straddle elements");
  static_assert(TW <= ROWS * RSL, "staging fits in the flux rows");
  static_assert(NQ > LA, "the lookahead is shorter than the quad sequence");
};

template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(WDims<N>::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void wmfma_stage_kernel(
    const double* __restrict__ u_in, double* __restrict__ out, double* __restrict__ res,
    const double* __restrict__ geo, const int32_t* __restrict__ fcode, const double* __restrict__ mat,
    const double* __restrict__ opf, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, double ca, double cb, double cdt, SrcArgs inc) {
  using D = WDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES, NF = D::NF,
                KS = D::KS, RSL = D::RSL, RT = D::RT, FIT = D::FIT, TC = D::TC, CPT = D::CPT,
                VB = D::VB, VR = D::VR, QV = D::QV, QF = D::QF, NQ = D::NQ, NTH = D::THREADS, LA = D::LA;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;
  constexpr int GPT = (GW + NTH - 1) / NTH;
  __shared__ __align__(16) double up_s[E * ES];            // field tile [e][f][n]
  __shared__ __align__(16) double gl[D::ROWS * RSL];       // flux rows [f E + e][fj]; later staging
  __shared__ double gt[GW];
  __shared__ __align__(16) double wmat[MAT ? E * 4 * dgh::kMatFace : 2];   // MAT: [e][f][A B C D]
  __shared__ int32_t fcb[2][E * 4];
  __shared__ uint8_t nbr_s[96 * NFP];
  __shared__ uint8_t fm_s[4 * NFP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int nt = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's column tile
  const int g4 = lane >> 4, li = lane & 15;
  // LDS slot of word q of a tile of the [K][6][Np] arrays (rows padded to NPP in LDS)
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NP), r = q - e * 6 * NP;
    if constexpr (NPP == NP) return e * ES + r;
    const int f = r / NP;
    return e * ES + f * NPP + (r - f * NP);
  };

  const int nwg = gridDim.x / kXcds;
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  for (int q = tid; q < 96 * NFP; q += NTH) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += NTH) fm_s[q] = uint8_t(fmask[q]);
  for (int q = tid; q < E * ES; q += NTH) up_s[q] = 0.0;
  __syncthreads();

  int tq = tid;
  asm volatile("" : "+v"(tq));
  doublex2 pu[CPT];
  double pg[GPT];
  double nup[FIT][6];
  int32_t pf = 0;
  double pm = 0.0, pw = 0.0;
  const size_t fc_last = size_t(K) * 4 - 1;
  const size_t chunk_last = size_t(K) * 6 * NP / 2 - 1;
  const doublex2* u2 = reinterpret_cast<const doublex2*>(u_in);
  // every load issued on every path, indices clamped into the arrays
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) pu[r] = u2[min(size_t(t) * TC + min(tid + r * NTH, TC - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * NTH, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  auto gather = [&](int t, const int32_t* fcv) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = min(tq + r * NTH, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const double* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NP + nn : size_t(e0 + e) * 6 * NP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NP];
    }
  };
  int par = 0;
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  gather(tile, fcb[0]);
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    const size_t tb = size_t(base) * 6 * NP;
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;

    // ---- tile into LDS
    if (full) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if ((r + 1) * NTH <= TC || c < TC) {
          if constexpr (NPP == NP) {
            *reinterpret_cast<doublex2*>(up_s + slot(2 * c)) = pu[r];
          } else {   // a chunk may straddle two padded rows
            up_s[slot(2 * c)] = pu[r].x;
            up_s[slot(2 * c + 1)] = pu[r].y;
          }
        }
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) up_s[slot(q)] = u_in[tb + q];
      if (MAT) {
        for (int q = tid; q < 2 * nel; q += NTH)
          up_s[(q >> 1) * ES + 6 * NPP + (q & 1)] = mat[(size_t(base) + (q >> 1)) * dgh::kMatStride + (q & 1)];
        for (int q = tid; q < 16 * nel; q += NTH)
          wmat[q] = mat[(size_t(base) + q / 16) * dgh::kMatStride + dgh::kMatFace + (q & 15)];
      }
      for (int q = tid; q < nel * G; q += NTH) gt[q] = geo[size_t(base) * G + q];
    }
    __syncthreads();

    // ---- face fluxes from the exterior traces gathered during the previous tile
    const int32_t* fc = fcb[par];
    __builtin_amdgcn_s_setprio(2);
    {
      if constexpr (NF > NF4)
        for (int q = tid; q < D::ROWS * (NF - NF4); q += NTH) {
          const int row = q / (NF - NF4);
          gl[row * RSL + NF4 + (q - row * (NF - NF4))] = 0.0;
        }
#pragma unroll
      for (int r = 0; r < FIT; ++r) {
        const int q = tq + r * NTH;
        if (q < nel * NF4) {
          const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
          const double* g = gt + e * G + dgh::kGeoNormal + 4 * f;
          const double nx = g[0], ny = g[1], nz = g[2], hs = 0.5 * g[3];
          const double* um = up_s + e * ES + fm_s[f * NFP + j];
          double m[6], d[6], w[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int c = 0; c < 6; ++c) m[c] = um[c * NPP];
          const int code = fc[e * 4 + f];
          if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
          face_jump(code, m, nup[r], d);
          if (MAT) {
            const doublex2 w01 = *reinterpret_cast<const doublex2*>(wmat + 16 * e + 4 * f);
            const doublex2 w23 = *reinterpret_cast<const doublex2*>(wmat + 16 * e + 4 * f + 2);
            w[0] = w01.x, w[1] = w01.y, w[2] = w23.x, w[3] = w23.y;
          }
          upwind_flux(MAT, nx, ny, nz, hs, w, d, gl + e * RSL + fj, E * RSL);
        }
      }
    }
    __syncthreads();

    // ---- contraction: this wave's column tile against the three row tiles; row tile t holds
    // rows 16 t + li, row = f E + e
    __builtin_amdgcn_s_setprio(3);
    // this wave's operator strip: quad q at bq[64 q] (four k-steps), single s at bs[64 s]; the
    // base address passes through an empty asm each tile, so the loads are not hoisted out of
    // the tile loop (the whole strip would then have to stay resident)
    const double* opw = opf + size_t(nt) * KS * 64;
    asm volatile("" : "+s"(opw));
    const doublex4* bq = reinterpret_cast<const doublex4*>(opw) + lane;
    const double* bs = opw + NQ * 256 + lane;
    doublex4 wb[LA];
#pragma unroll
    for (int i = 0; i < LA; ++i) wb[i] = bq[64 * i];
    double w1[3 * VR > 0 ? 3 * VR : 1];
#pragma unroll
    for (int i = 0; i < 3 * VR; ++i) w1[i] = bs[64 * i];
    // the next tile's fields and geometry, issued behind the first operator quads
    prefetch(nxt);
    doublex4 acc[RT];
    {
      double pc[RT][3], qc[RT][3];   // operand = pc[mu] V_c + qc[mu] V_b
      const double* vc[RT];
      const double* vb[RT];
      const double* fl[RT];
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        acc[t] = doublex4{0.0, 0.0, 0.0, 0.0};
        const int row = 16 * t + li;
        const int f = row / E, e = row - f * E;
        const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
        const int srcf = f < 3 ? 3 : 0;            // H feeds the E rows, E the H rows
        const double sg = f < 3 ? 1.0 : -1.0;
        const double* cm = gt + e * G;
        const double sm = MAT ? sg * up_s[e * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          pc[t][mu] = sm * cm[3 * mu + b];
          qc[t][mu] = -sm * cm[3 * mu + c];
        }
        vc[t] = up_s + e * ES + (srcf + c) * NPP;
        vb[t] = up_s + e * ES + (srcf + b) * NPP;
        fl[t] = gl + row * RSL + 4 * g4;
      }
      auto ld4 = [](const double* p) __attribute__((always_inline)) {
        const doublex2 lo = *reinterpret_cast<const doublex2*>(p);
        const doublex2 hi = *reinterpret_cast<const doublex2*>(p + 2);
        return doublex4{lo.x, lo.y, hi.x, hi.y};
      };
      // operator quad q: the one loaded LA quads ago; its buffer takes quad q + LA
      auto quad = [&](int q) __attribute__((always_inline)) {
        const doublex4 w = wb[q % LA];
        if (q + LA < NQ) wb[q % LA] = bq[64 * (q + LA)];
        return w;
      };
#pragma unroll
      for (int jb = 0; jb < VB; ++jb) {
        doublex4 xc[RT], xb[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          xc[t] = ld4(vc[t] + 16 * jb + 4 * g4);
          xb[t] = ld4(vb[t] + 16 * jb + 4 * g4);
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const doublex4 w = quad(3 * jb + mu);
#pragma unroll
          for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int t = 0; t < RT; ++t)
              acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(pc[t][mu] * xc[t][s] + qc[t][mu] * xb[t][s], w[s],
                                                            acc[t], 0, 0, 0);
        }
      }
#pragma unroll
      for (int fb = 0; fb < QF; ++fb) {
        doublex4 xf[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) xf[t] = ld4(fl[t] + 16 * fb);
        const doublex4 w = quad(QV + fb);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int t = 0; t < RT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xf[t][s], w[s], acc[t], 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < VR; ++r) {
        double xc1[RT], xb1[RT];
#pragma unroll
        for (int t = 0; t < RT; ++t) {
          xc1[t] = vc[t][16 * VB + 4 * r + g4];
          xb1[t] = vb[t][16 * VB + 4 * r + g4];
        }
#pragma unroll
        for (int mu = 0; mu < 3; ++mu)
#pragma unroll
          for (int t = 0; t < RT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(pc[t][mu] * xc1[t] + qc[t][mu] * xb1[t], w1[3 * r + mu],
                                                          acc[t], 0, 0, 0);
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // the next tile's exterior traces, then this tile's residual
    gather(nxt, fcb[more ? par ^ 1 : par]);
    doublex2 rs[CPT];
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r)
        rs[r] = __builtin_nontemporal_load(reinterpret_cast<const doublex2*>(res) +
                                           min(size_t(tile) * TC + min(tid + r * NTH, TC - 1), chunk_last));
    }
    __syncthreads();   // flux rows are read: reuse them for the staging

    // ---- stage the right-hand side [e][f][n] contiguously (nodes >= Np are the padding of
    // the last column tile)
    double* stage = gl;
    const int col = 16 * nt + li;
    if (col < NP) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * t + g4 + 4 * i;
          const int f = row / E, e = row - f * E;
          stage[(e * 6 + f) * NP + col] = acc[t][i];
        }
    }
    __syncthreads();

    // ---- update and write out, 16-byte chunks
    if (full) {
      doublex2* o2 = reinterpret_cast<doublex2*>(out + tb);
      doublex2* r2 = reinterpret_cast<doublex2*>(res + tb);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if ((r + 1) * NTH <= TC || c < TC) {
          const doublex2 h = reinterpret_cast<const doublex2*>(stage)[c];
          if (STAGE) {
            doublex2 u;
            if constexpr (NPP == NP) {
              u = *reinterpret_cast<const doublex2*>(up_s + slot(2 * c));
            } else {
              u = doublex2{up_s[slot(2 * c)], up_s[slot(2 * c + 1)]};
            }
            const doublex2 rv = doublex2{ca * rs[r].x + cdt * h.x, ca * rs[r].y + cdt * h.y};
            __builtin_nontemporal_store(rv, r2 + c);
            __builtin_nontemporal_store(doublex2{u.x + cb * rv.x, u.y + cb * rv.y}, o2 + c);
          } else {
            o2[c] = h;
          }
        }
      }
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) {
        const double h = stage[q];
        if (STAGE) {
          const double rv = ca * res[tb + q] + cdt * h;
          res[tb + q] = rv;
          out[tb + q] = up_s[slot(q)] + cb * rv;
        } else {
          out[tb + q] = h;
        }
      }
    }
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();   // the next tile overwrites up_s, gt, fcb and gl
  }
}

// ---------------------------------------------------------------------------------------
// Split-BF16 form of the FP32 contraction (N = 5, 6, 7): each value x of the operand and of
// the operator is carried as x_hi + x_lo, x_hi = bf16(x), x_lo = bf16(x - x_hi), and a
// product is taken as x_hi y_hi + x_hi y_lo + x_lo y_hi (three v_mfma_f32_16x16x32_bf16 per
// 32-deep k-block, FP32 accumulation). Per product the error is about 3 * 2^-18 |x y| (the
// dropped x_lo y_lo and the two splitting residuals), so the result carries about 1e-5 of
// the absolute sum of its terms; the state, the fluxes and the RK update stay FP32.
//
// k-axis of one element row: [D_r | D_s | D_t] blocks of NP8 = roundup(Np, 8) nodes, then the
// face block of NF8 = roundup(4 Nfp, 8) face nodes, zero-padded to KD = roundup(., 32). Lane
// (li, g4) of a 16x16x32 step holds k-values 32 b + 8 g4 .. + 7 of row li, which lie in one
// block. The operator is split once on the host and kept in VGPRs (8 per k-block and lane);
// the operand is formed once per tile, for all column tiles, and stored split in LDS:
//   volume columns (mu, n): pc[mu] V_c[n] + qc[mu] V_b[n] (the contravariant flux, as in the
//   FP32 kernels), face columns: the Fscale-scaled upwind flux, written by the flux phase.
// Tile, waves and memory phases follow the FP32 kernel for these orders: 8 elements (three
// 16-row tiles), one wave per 16-node column tile.
template <int N>
struct BDims {
  static constexpr int Np = Dims<N>::Np, Nfp = Dims<N>::Nfp, Nf4 = Dims<N>::Nf4;
  static constexpr int E = 8, ROWS = 6 * E, RT = ROWS / 16;
  static constexpr int NT = (Np + 15) / 16, THREADS = 64 * NT;
  static constexpr int NPP = Np;                      // field rows (Np % 4 == 0 at these orders)
  static constexpr int ES = 6 * NPP + 4;
  static constexpr int NP8 = (Np + 7) / 8 * 8, KV = 3 * NP8;
  static constexpr int NF8 = (Nf4 + 7) / 8 * 8;
  static constexpr int KD = (KV + NF8 + 31) / 32 * 32, KB = KD / 32;
  static constexpr int AS = KD + 8;                   // operand row stride (bf16), rows 16 B aligned
  static constexpr int VG = KV / 8;                   // 8-column volume groups per row
  static constexpr int TW = E * 6 * Np, TW4 = TW / 4;
  static constexpr int CPT = (TW4 + THREADS - 1) / THREADS;
  static constexpr int FIT = (E * Nf4 + THREADS - 1) / THREADS;
  static constexpr int OPW = NT * KB * 64 * 16;       // operator table, bf16 words
  static_assert(Np % 4 == 0, "16-byte chunks of a tile map to the LDS rows");
  static_assert(2 * TW <= ROWS * AS, "staging fits in the low-part array");
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(BDims<N>::THREADS) __attribute__((amdgpu_waves_per_eu(2, 2))) void bmfma_stage_kernel(
    const float* __restrict__ u_in, float* __restrict__ out, float* __restrict__ res,
    const float* __restrict__ geo, const int32_t* __restrict__ fcode, const float* __restrict__ mat,
    const uint16_t* __restrict__ opb, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, float ca, float cb, float cdt, SrcArgs inc) {
  using D = BDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES, RT = D::RT,
                NP8 = D::NP8, KV = D::KV, KD = D::KD, KB = D::KB, AS = D::AS, VG = D::VG, TW4 = D::TW4,
                CPT = D::CPT, FIT = D::FIT, NTH = D::THREADS;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;
  constexpr int GPT = (GW + NTH - 1) / NTH;
  __shared__ __align__(16) float up_s[E * ES];             // field tile [e][f][n]
  __shared__ __align__(16) __bf16 ahi[D::ROWS * AS];       // operand, high parts [f E + e][k]
  __shared__ __align__(16) __bf16 alo[D::ROWS * AS];       // operand, low parts; later staging
  __shared__ float gt[GW];
  __shared__ __align__(16) float wmat[MAT ? E * 4 * dgh::kMatFace : 4];
  __shared__ int32_t fcb[2][E * 4];
  __shared__ uint8_t nbr_s[96 * NFP];
  __shared__ uint8_t fm_s[4 * NFP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int nt = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's column tile
  const int g4 = lane >> 4, li = lane & 15;
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NP);
    return e * ES + (q - e * 6 * NP);
  };
  auto split = [](float x, __bf16& h, __bf16& l) __attribute__((always_inline)) {
    h = __bf16(x);
    l = __bf16(x - float(h));
  };

  const int nwg = gridDim.x / kXcds;
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  // once per workgroup: this wave's operator (high and low parts per k-block), node tables, the
  // zero padding of the operand rows (face columns past 4 Nfp; never written afterwards)
  bf16x8 bh[KB], bl[KB];
  {
    const bf16x8* src = reinterpret_cast<const bf16x8*>(opb) + size_t(nt) * KB * 64 * 2 + 2 * lane;
#pragma unroll
    for (int b = 0; b < KB; ++b) {
      bh[b] = src[b * 128];
      bl[b] = src[b * 128 + 1];
    }
  }
  for (int q = tid; q < 96 * NFP; q += NTH) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += NTH) fm_s[q] = uint8_t(fmask[q]);
  for (int q = tid; q < D::ROWS * AS; q += NTH) {
    ahi[q] = __bf16(0.f);
    alo[q] = __bf16(0.f);
  }

  int tq = tid;
  asm volatile("" : "+v"(tq));
  floatx4 pu[CPT];
  float pg[GPT];
  float nup[FIT][6];
  int32_t pf = 0;
  float pm = 0.f, pw = 0.f;
  const size_t fc_last = size_t(K) * 4 - 1;
  const size_t chunk_last = size_t(K) * 6 * NP / 4 - 1;
  const floatx4* u4 = reinterpret_cast<const floatx4*>(u_in);
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) pu[r] = u4[min(size_t(t) * TW4 + min(tid + r * NTH, TW4 - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * NTH, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  auto gather = [&](int t, const int32_t* fcv) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = min(tq + r * NTH, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const float* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NP + nn : size_t(e0 + e) * 6 * NP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NP];
    }
  };
  int par = 0;
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    const size_t tb = size_t(base) * 6 * NP;
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;

    if (full) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int q = tid + r * NTH;
        if (q < TW4) *reinterpret_cast<floatx4*>(up_s + slot(4 * q)) = pu[r];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) up_s[slot(q)] = u_in[tb + q];
      if (MAT) {
        for (int q = tid; q < 2 * nel; q += NTH)
          up_s[(q >> 1) * ES + 6 * NPP + (q & 1)] = mat[(size_t(base) + (q >> 1)) * dgh::kMatStride + (q & 1)];
        for (int q = tid; q < 16 * nel; q += NTH)
          wmat[q] = mat[(size_t(base) + q / 16) * dgh::kMatStride + dgh::kMatFace + (q & 15)];
      }
      for (int q = tid; q < nel * G; q += NTH) gt[q] = geo[size_t(base) * G + q];
    }
    __syncthreads();

    // ---- face fluxes, written split into the face columns of the operand rows; the face
    // padding columns (their operator columns are zero) are cleared again, since the staging
    // of the previous tile wrote over the low parts
    const int32_t* fc = fcb[par];
    gather(tile, fc);
    if constexpr (KD > KV + NF4)
      for (int q = tid; q < D::ROWS * (KD - KV - NF4); q += NTH) {
        const int row = q / (KD - KV - NF4), col = KV + NF4 + (q - row * (KD - KV - NF4));
        ahi[row * AS + col] = __bf16(0.f);
        alo[row * AS + col] = __bf16(0.f);
      }
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = tq + r * NTH;
      if (q < nel * NF4) {
        const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
        const float* g = gt + e * G + dgh::kGeoNormal + 4 * f;
        const float nx = g[0], ny = g[1], nz = g[2], hs = 0.5f * g[3];
        const float* um = up_s + e * ES + fm_s[f * NFP + j];
        float m[6], d[6], w[4] = {0.f, 0.f, 0.f, 0.f}, fl[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) m[c] = um[c * NPP];
        const int code = fc[e * 4 + f];
        if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
        face_jump(code, m, nup[r], d);
        if (MAT) {
          const floatx4 wv = *reinterpret_cast<const floatx4*>(wmat + 16 * e + 4 * f);
          w[0] = wv.x, w[1] = wv.y, w[2] = wv.z, w[3] = wv.w;
        }
        upwind_flux(MAT, nx, ny, nz, hs, w, d, fl, 1);
#pragma unroll
        for (int c = 0; c < 6; ++c) split(fl[c], ahi[(c * E + e) * AS + KV + fj], alo[(c * E + e) * AS + KV + fj]);
      }
    }
    // ---- volume columns: the contravariant flux, eight nodes of one direction per item
    for (int q = tid; q < D::ROWS * VG; q += NTH) {
      const int row = q / VG, grp = q - row * VG;
      const int f = row / E, e = row - f * E;
      const int mu = (8 * grp) / NP8, n0 = 8 * grp - mu * NP8;
      const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
      const int srcf = f < 3 ? 3 : 0;
      const float sg = f < 3 ? 1.f : -1.f;
      const float sm = MAT ? sg * up_s[e * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
      const float pc = sm * gt[e * G + 3 * mu + b], qc = -sm * gt[e * G + 3 * mu + c];
      const float* vc = up_s + e * ES + (srcf + c) * NPP + n0;
      const float* vb = up_s + e * ES + (srcf + b) * NPP + n0;
      const floatx4 c0 = *reinterpret_cast<const floatx4*>(vc), c1 = *reinterpret_cast<const floatx4*>(vc + 4);
      const floatx4 b0 = *reinterpret_cast<const floatx4*>(vb), b1 = *reinterpret_cast<const floatx4*>(vb + 4);
      const float xv[8] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w};
      const float yv[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
      bf16x8 h, l;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        // nodes past Np (NP8 > Np) read the next row or the row padding: finite, and their
        // operator columns are zero; they are stored as zero all the same
        const float gv = n0 + jj < NP ? pc * xv[jj] + qc * yv[jj] : 0.f;
        __bf16 hh, ll;
        split(gv, hh, ll);
        h[jj] = hh;
        l[jj] = ll;
      }
      *reinterpret_cast<bf16x8*>(ahi + row * AS + 8 * grp) = h;
      *reinterpret_cast<bf16x8*>(alo + row * AS + 8 * grp) = l;
    }
    floatx4 rs4[CPT];
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r)
        rs4[r] = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(res) +
                                            min(size_t(tile) * TW4 + min(tid + r * NTH, TW4 - 1), chunk_last));
    }
    prefetch(nxt);
    __syncthreads();

    // ---- contraction: three products per 32-deep k-block
    floatx4 acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < KB; ++b) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const int o = (16 * t + li) * AS + 32 * b + 8 * g4;
        const bf16x8 xh = *reinterpret_cast<const bf16x8*>(ahi + o);
        const bf16x8 xl = *reinterpret_cast<const bf16x8*>(alo + o);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, bh[b], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bl[b], acc[t], 0, 0, 0);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, bh[b], acc[t], 0, 0, 0);
      }
    }
    __syncthreads();   // the operand is read: reuse its low parts for the staging

    // ---- stage the right-hand side [e][f][n]: lane (li, g4), register i = row 16 t + 4 g4 + i
    float* stage = reinterpret_cast<float*>(alo);
    const int col = 16 * nt + li;
    if (col < NP) {
#pragma unroll
      for (int t = 0; t < RT; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = 16 * t + 4 * g4 + i;
          const int f = row / E, e = row - f * E;
          stage[(e * 6 + f) * NP + col] = acc[t][i];
        }
    }
    __syncthreads();

    if (full) {
      floatx4* o4 = reinterpret_cast<floatx4*>(out + tb);
      floatx4* r4 = reinterpret_cast<floatx4*>(res + tb);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int q = tid + r * NTH;
        if (q < TW4) {
          const floatx4 h = reinterpret_cast<const floatx4*>(stage)[q];
          if (STAGE) {
            const floatx4 u = *reinterpret_cast<const floatx4*>(up_s + slot(4 * q));
            const floatx4 rv = ca * rs4[r] + cdt * h;
            __builtin_nontemporal_store(rv, r4 + q);
            __builtin_nontemporal_store(u + cb * rv, o4 + q);
          } else {
            o4[q] = h;
          }
        }
      }
    } else {
      for (int q = tid; q < nel * 6 * NP; q += NTH) {
        const float h = stage[q];
        if (STAGE) {
          const float rv = ca * res[tb + q] + cdt * h;
          res[tb + q] = rv;
          out[tb + q] = up_s[slot(q)] + cb * rv;
        } else {
          out[tb + q] = h;
        }
      }
    }
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------------------
// FP32 contraction on small tiles (serves N = 3): the structure of the FP64 kernel above with
// the FP32 matrix instructions. A tile of 8 elements has 48 field-major (field, element) rows;
// wave t computes row tile t (rows 16 t .. 16 t + 15) against all column tiles on
// v_mfma_f32_16x16x4f32 and the Np mod 16 tail columns on v_mfma_f32_4x4x1f32 (its 16 blocks
// read as (k-group, row quad) pairs from the same operand register, a cross-lane sum over the
// k-groups at the end, as in the 16-element kernel), so the three waves carry equal matrix
// work; LDS holds the fields, the fluxes and the operator (three workgroups per CU). The field
// arrays keep their padded rows (roundup(Np, 4) words, pad words zero); the next tile's loads
// are issued during the contraction; issue priorities; nontemporal residual and state I/O.
// Measured on 384,000 tets: N = 3 212.3 us per stage against 259.0 us on the 16-element
// kernel; at N = 4 it is slower (483 against 422 us), so N = 4 keeps the 16-element kernel.
template <int N>
struct SDims {
  using M = MDims<N>;
  static constexpr int Np = M::Np, Nfp = M::Nfp, Nf4 = M::Nf4;
  static constexpr int E = 8;                         // elements per tile
  static constexpr int WAVES = 6 * E / 16, THREADS = 64 * WAVES;
  static constexpr int NPP = M::NPP;                  // padded row of the field arrays
  static constexpr int ES = 6 * NPP + 4;              // element stride in LDS (= 4 mod 8 words)
  static constexpr int NF = M::NF, RSL = NF + 4;      // flux row stride (= 4 mod 8 words)
  static constexpr int KS = M::KS, VB = M::VB, VR = M::VR, QV = M::QV, QF = M::QF, NQ = M::NQ;
  static constexpr int NT = M::NT, TAIL = M::TAIL;
  static constexpr int PC = NPP / 4;                  // 16-byte chunks per padded row
  static constexpr int LAST = Np - 4 * (PC - 1);      // field words in the last chunk of a row
  static constexpr int TW = E * 6 * NPP;
  static constexpr int TC = TW / 4;                   // 16-byte chunks per tile
  static constexpr int CPT = (TC + THREADS - 1) / THREADS;
  static constexpr int FIT = (E * Nf4 + THREADS - 1) / THREADS;
  static constexpr int OPC = M::OPC;
  static_assert(TAIL > 0 && TAIL <= 4, "one 4-column tail block");
  static_assert(E * ES <= 6 * E * RSL, "staging fits in the flux rows");
};

template <int N, bool STAGE, bool MAT, bool SRC>
__global__ __launch_bounds__(SDims<N>::THREADS) __attribute__((amdgpu_waves_per_eu(3, 3))) void smfma_stage_kernel(
    const float* __restrict__ u_in, float* __restrict__ out, float* __restrict__ res,
    const float* __restrict__ geo, const int32_t* __restrict__ fcode, const float* __restrict__ mat,
    const float* __restrict__ opf, const int32_t* __restrict__ fmask,
    const int32_t* __restrict__ nbrnode, int K, int ntiles, float ca, float cb, float cdt, SrcArgs inc) {
  using D = SDims<N>;
  constexpr int NP = D::Np, NFP = D::Nfp, NF4 = D::Nf4, E = D::E, NPP = D::NPP, ES = D::ES, NF = D::NF,
                KS = D::KS, RSL = D::RSL, NT = D::NT, TAIL = D::TAIL, FIT = D::FIT, TC = D::TC, CPT = D::CPT,
                VB = D::VB, VR = D::VR, QV = D::QV, QF = D::QF, NQ = D::NQ, NTH = D::THREADS, PC = D::PC,
                LAST = D::LAST;
  constexpr int G = dgh::kGeoStride;
  constexpr int GW = E * G;
  constexpr int GPT = (GW + NTH - 1) / NTH;
  __shared__ __align__(16) float up_s[E * ES];             // field tile [e][f][NPP]
  __shared__ __align__(16) float gl[6 * E * RSL];          // flux rows [f E + e][fj]; later staging
  __shared__ __align__(16) float bfs[NT * KS * 64];        // operator fragments
  __shared__ __align__(16) float tops[KS * 16];            // tail operator (k-group, column)
  __shared__ float gt[GW];
  __shared__ __align__(16) float wmat[MAT ? E * 4 * dgh::kMatFace : 4];   // MAT: [e][f][A B C D]
  __shared__ int32_t fcb[2][E * 4];
  __shared__ uint8_t nbr_s[96 * NFP];
  __shared__ uint8_t fm_s[4 * NFP];

  const int tid = threadIdx.x, lane = tid & 63;
  const int fw = __builtin_amdgcn_readfirstlane(tid >> 6);   // this wave's 16-row tile
  const int g4 = lane >> 4, li = lane & 15;
  auto slot = [](int q) __attribute__((always_inline)) {
    const int e = q / (6 * NPP);
    return e * ES + (q - e * 6 * NPP);
  };
  auto pad_zero = [](int c, floatx4 v) __attribute__((always_inline)) {   // pad words of a row
    if (LAST < 4 && c % PC == PC - 1) {
      if (LAST <= 3) v.w = 0.f;
      if (LAST <= 2) v.z = 0.f;
      if (LAST <= 1) v.y = 0.f;
    }
    return v;
  };

  const int nwg = gridDim.x / kXcds;
  const int xcd = blockIdx.x % kXcds, wj = blockIdx.x / kXcds;
  const int TX = (ntiles + kXcds - 1) / kXcds;
  const int tend = min(ntiles, (xcd + 1) * TX);
  int tile = xcd * TX + wj;
  if (tile >= tend) return;

  for (int q = tid; q < NT * KS * 64; q += NTH) bfs[q] = opf[q];
  for (int q = tid; q < KS * 16; q += NTH) tops[q] = opf[NT * KS * 64 + q];
  for (int q = tid; q < 96 * NFP; q += NTH) nbr_s[q] = uint8_t(nbrnode[q]);
  for (int q = tid; q < 4 * NFP; q += NTH) fm_s[q] = uint8_t(fmask[q]);
  for (int q = tid; q < E * ES; q += NTH) up_s[q] = 0.f;
  __syncthreads();

  int tq = tid;
  if (MAT) asm volatile("" : "+v"(tq));
  floatx4 pu[CPT];
  float pg[GPT];
  float nup[FIT][6];
  int32_t pf = 0;
  float pm = 0.f, pw = 0.f;
  const size_t fc_last = size_t(K) * 4 - 1;
  const size_t chunk_last = size_t(K) * 6 * NPP / 4 - 1;
  const floatx4* u4 = reinterpret_cast<const floatx4*>(u_in);
  auto prefetch = [&](int t) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < CPT; ++r) pu[r] = u4[min(size_t(t) * TC + min(tid + r * NTH, TC - 1), chunk_last)];
#pragma unroll
    for (int r = 0; r < GPT; ++r)
      pg[r] = geo[min(size_t(t) * GW + min(tid + r * NTH, GW - 1), size_t(K) * G - 1)];
    if (MAT) {
      const int q = min(tid, 2 * E - 1);
      const size_t e = min(size_t(t) * E + q / 2, size_t(K) - 1);
      pm = mat[e * dgh::kMatStride + (q & 1)];
      const int qw = min(tid, 16 * E - 1);
      const size_t ew = min(size_t(t) * E + qw / 16, size_t(K) - 1);
      pw = mat[ew * dgh::kMatStride + dgh::kMatFace + (qw & 15)];
    }
    pf = fcode[min(size_t(t + nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];
  };
  auto gather = [&](int t, const int32_t* fcv) __attribute__((always_inline)) {
    const int e0 = t * E, nl = min(E, K - e0);
#pragma unroll
    for (int r = 0; r < FIT; ++r) {
      const int q = min(tq + r * NTH, nl * NF4 - 1);
      const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
      const int code = fcv[e * 4 + f];
      const int ci = code >= 0 ? code : 0;
      const int nn = nbr_s[((f * 4 + (ci & 3)) * 6 + ((ci >> 2) & 7)) * NFP + j];
      const float* p = u_in + (code >= 0 ? size_t(ci >> 5) * 6 * NPP + nn : size_t(e0 + e) * 6 * NPP);
#pragma unroll
      for (int c = 0; c < 6; ++c) nup[r][c] = p[c * NPP];
    }
  };
  int par = 0;
  if (tid < E * 4) {
    fcb[0][tid] = fcode[min(size_t(tile) * E * 4 + tid, fc_last)];
    fcb[1][tid] = fcode[min(size_t(tile + nwg) * E * 4 + tid, fc_last)];
  }
  __syncthreads();
  gather(tile, fcb[0]);
  prefetch(tile);
  pf = fcode[min(size_t(tile + 2 * nwg) * E * 4 + min(tid, E * 4 - 1), fc_last)];

  for (; tile < tend; tile += nwg) {
    const int base = tile * E;
    const int nel = min(E, K - base);
    const bool full = nel == E;
    const size_t tb = size_t(base) * 6 * NPP;
    const bool more = tile + nwg < tend;
    const int nxt = more ? tile + nwg : tile;

    // ---- tile into LDS
    if (full) {
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if ((r + 1) * NTH <= TC || c < TC) *reinterpret_cast<floatx4*>(up_s + slot(4 * c)) = pu[r];
      }
#pragma unroll
      for (int r = 0; r < GPT; ++r) {
        const int q = tid + r * NTH;
        if (q < GW) gt[q] = pg[r];
      }
      if (MAT && tid < 2 * E) up_s[(tid >> 1) * ES + 6 * NPP + (tid & 1)] = pm;
      if (MAT && tid < 16 * E) wmat[tid] = pw;
    } else {
      for (int q = tid; q < nel * 6 * NPP; q += NTH) up_s[slot(q)] = u_in[tb + q];
      if (MAT) {
        for (int q = tid; q < 2 * nel; q += NTH)
          up_s[(q >> 1) * ES + 6 * NPP + (q & 1)] = mat[(size_t(base) + (q >> 1)) * dgh::kMatStride + (q & 1)];
        for (int q = tid; q < 16 * nel; q += NTH)
          wmat[q] = mat[(size_t(base) + q / 16) * dgh::kMatStride + dgh::kMatFace + (q & 15)];
      }
      for (int q = tid; q < nel * G; q += NTH) gt[q] = geo[size_t(base) * G + q];
    }
    __syncthreads();

    // ---- face fluxes from the exterior traces gathered during the previous tile
    const int32_t* fc = fcb[par];
    __builtin_amdgcn_s_setprio(2);
    {
      if constexpr (NF > NF4)
        for (int q = tid; q < 6 * E * (NF - NF4); q += NTH) {
          const int row = q / (NF - NF4);
          gl[row * RSL + NF4 + (q - row * (NF - NF4))] = 0.f;
        }
#pragma unroll
      for (int r = 0; r < FIT; ++r) {
        const int q = tq + r * NTH;
        if (q < nel * NF4) {
          const int e = q / NF4, fj = q - e * NF4, f = fj / NFP, j = fj - f * NFP;
          const float* g = gt + e * G + dgh::kGeoNormal + 4 * f;
          const float nx = g[0], ny = g[1], nz = g[2], hs = 0.5f * g[3];
          const float* um = up_s + e * ES + fm_s[f * NFP + j];
          float m[6], d[6], w[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int c = 0; c < 6; ++c) m[c] = um[c * NPP];
          const int code = fc[e * 4 + f];
          if (SRC && code <= dgh::kFaceScatter0) add_incident(inc, code, j, NFP, m);
          face_jump(code, m, nup[r], d);
          if (MAT) {
            const floatx4 wv = *reinterpret_cast<const floatx4*>(wmat + 16 * e + 4 * f);
            w[0] = wv.x, w[1] = wv.y, w[2] = wv.z, w[3] = wv.w;
          }
          upwind_flux(MAT, nx, ny, nz, hs, w, d, gl + e * RSL + fj, E * RSL);
        }
      }
    }
    __syncthreads();
    __builtin_amdgcn_s_setprio(0);
    floatx4 rs[CPT];
    if (STAGE) {
#pragma unroll
      for (int r = 0; r < CPT; ++r)
        rs[r] = __builtin_nontemporal_load(reinterpret_cast<const floatx4*>(res) +
                                           min(size_t(tile) * TC + min(tid + r * NTH, TC - 1), chunk_last));
    }
    // the next tile's fields and geometry, then its exterior traces
    prefetch(nxt);
    gather(nxt, fcb[more ? par ^ 1 : par]);

    // ---- contraction of row tile fw: row 16 fw + li = (field f, element el)
    __builtin_amdgcn_s_setprio(3);
    floatx4 acc[NT], tacc = floatx4{0.f, 0.f, 0.f, 0.f};
    {
      const int row = 16 * fw + li, f = row / E, el = row - f * E;
      const int a = f % 3, b = (a + 1) % 3, c = (a + 2) % 3;
      const int srcf = f < 3 ? 3 : 0;            // H feeds the E rows, E the H rows
      const float sg = f < 3 ? 1.f : -1.f;
      const float* cm = gt + el * G;
      const float sm = MAT ? sg * up_s[el * ES + 6 * NPP + (f < 3 ? 0 : 1)] : sg;
      float pc[3], qc[3];   // operand = pc[mu] V_c + qc[mu] V_b
#pragma unroll
      for (int mu = 0; mu < 3; ++mu) {
        pc[mu] = sm * cm[3 * mu + b];
        qc[mu] = -sm * cm[3 * mu + c];
      }
      const float* vc = up_s + el * ES + (srcf + c) * NPP;
      const float* vb = up_s + el * ES + (srcf + b) * NPP;
      const float* fl = gl + row * RSL + 4 * g4;
#pragma unroll
      for (int t = 0; t < NT; ++t) acc[t] = floatx4{0.f, 0.f, 0.f, 0.f};
      const floatx4* bq = reinterpret_cast<const floatx4*>(bfs) + lane;   // quad q of tile t: bq[(t KS + 4 q) 16]
      const float* bs = bfs + NQ * 256 + lane;                             // single s of tile t: bs[t KS 64 + 64 s]
      const int tl = 4 * g4 + (li & 3);
      const floatx4* tq4 = reinterpret_cast<const floatx4*>(tops) + tl;   // tail quad q: tq4[16 q]
      const float* ts1 = tops + NQ * 64 + tl;                              // tail single s: ts1[16 s]
      auto step = [&](float av, const floatx4 (&w)[NT], const floatx4& z, int s) __attribute__((always_inline)) {
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, w[t][s], acc[t], 0, 0, 0);
        tacc = __builtin_amdgcn_mfma_f32_4x4x1f32(av, z[s], tacc, 0, 0, 0);
      };
#pragma unroll
      for (int jb = 0; jb < VB; ++jb) {
        const floatx4 xc = *reinterpret_cast<const floatx4*>(vc + 16 * jb + 4 * g4);
        const floatx4 xb = *reinterpret_cast<const floatx4*>(vb + 16 * jb + 4 * g4);
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const int q = 3 * jb + mu;
          floatx4 w[NT];
#pragma unroll
          for (int t = 0; t < NT; ++t) w[t] = bq[(t * KS) * 16 + 64 * q];
          const floatx4 z = tq4[16 * q];
#pragma unroll
          for (int s = 0; s < 4; ++s) step(pc[mu] * xc[s] + qc[mu] * xb[s], w, z, s);
        }
      }
#pragma unroll
      for (int fb = 0; fb < QF; ++fb) {
        const int q = QV + fb;
        const floatx4 xf = *reinterpret_cast<const floatx4*>(fl + 16 * fb);
        floatx4 w[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) w[t] = bq[(t * KS) * 16 + 64 * q];
        const floatx4 z = tq4[16 * q];
#pragma unroll
        for (int s = 0; s < 4; ++s) step(xf[s], w, z, s);
      }
#pragma unroll
      for (int r = 0; r < VR; ++r) {
        const float xc1 = vc[16 * VB + 4 * r + g4];   // columns >= Np read the zero padding
        const float xb1 = vb[16 * VB + 4 * r + g4];
#pragma unroll
        for (int mu = 0; mu < 3; ++mu) {
          const int sgl = 3 * r + mu;
          const float av = pc[mu] * xc1 + qc[mu] * xb1;
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bs[t * KS * 64 + 64 * sgl], acc[t], 0, 0, 0);
          tacc = __builtin_amdgcn_mfma_f32_4x4x1f32(av, ts1[16 * sgl], tacc, 0, 0, 0);
        }
      }
    }
    __builtin_amdgcn_s_setprio(0);
    // tail: sum the partial results of the four k-groups (lanes li, li + 16, li + 32, li + 48)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float v = tacc[i];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      tacc[i] = v;
    }
    __syncthreads();   // flux rows are read: reuse them for the staging

    // ---- stage the right-hand side [e][f][NPP] (laid out like up_s). 16x16x4 result: lane
    // (li, g4), register i = row 16 fw + 4 g4 + i, node 16 t + li. Tail (lanes g4 = 0): lane li,
    // register i = row 16 fw + 4 (li / 4) + i, node 16 NT + li mod 4.
    float* stage = gl;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * fw + 4 * g4 + i, f = row / E, el = row - f * E;
        stage[el * ES + f * NPP + 16 * t + li] = acc[t][i];
      }
    if (g4 == 0 && (li & 3) < TAIL) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = 16 * fw + 4 * (li >> 2) + i, f = row / E, el = row - f * E;
        stage[el * ES + f * NPP + 16 * NT + (li & 3)] = tacc[i];
      }
    }
    __syncthreads();

    // ---- update and write out, 16-byte chunks (pad words written as zero)
    if (full) {
      floatx4* o4 = reinterpret_cast<floatx4*>(out + tb);
      floatx4* r4 = reinterpret_cast<floatx4*>(res + tb);
#pragma unroll
      for (int r = 0; r < CPT; ++r) {
        const int c = tid + r * NTH;
        if ((r + 1) * NTH <= TC || c < TC) {
          const int o = slot(4 * c);
          const floatx4 h = *reinterpret_cast<const floatx4*>(stage + o);
          if (STAGE) {
            const floatx4 u = *reinterpret_cast<const floatx4*>(up_s + o);
            const floatx4 rv = pad_zero(c, ca * rs[r] + cdt * h);
            __builtin_nontemporal_store(rv, r4 + c);
            __builtin_nontemporal_store(u + cb * rv, o4 + c);
          } else {
            o4[c] = pad_zero(c, h);
          }
        }
      }
    } else {
      for (int q = tid; q < nel * 6 * NPP; q += NTH) {
        const bool node = q % NPP < NP;   // pad words stay zero
        const float h = node ? stage[slot(q)] : 0.f;
        if (STAGE) {
          const float rv = node ? ca * res[tb + q] + cdt * h : 0.f;
          res[tb + q] = rv;
          out[tb + q] = up_s[slot(q)] + cb * rv;
        } else {
          out[tb + q] = h;
        }
      }
    }
    if (tile + 2 * nwg < tend && tid < E * 4) fcb[par][tid] = pf;
    par ^= 1;
    __syncthreads();   // the next tile overwrites up_s, gt, fcb and gl
  }
}

// Resident workgroups for the persistent grid: CUs x workgroups per CU, a multiple of the XCD
// count (queried once per kernel and device: the template argument is the kernel itself, so
// every kernel keeps its own count).
template <auto Kern>
int persistent_grid(int threads, int ntiles) {
  // resident workgroups of this kernel, per device (the current one); a benign race only
  // recomputes the same value
  static std::atomic<int> cached[kMaxDevices];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = -1;
  int res = dev >= 0 ? cached[dev].load(std::memory_order_relaxed) : 0;
  if (!res) {
    int cus = 0, per = 0;
    if (dev < 0 || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, Kern, threads, 0) != hipSuccess || per < 1)
      per = 1, cus = 256;
    res = ((cus * per + kXcds - 1) / kXcds) * kXcds;
    if (dev >= 0) cached[dev].store(res, std::memory_order_relaxed);
  }
  const int want = ((ntiles + kXcds - 1) / kXcds) * kXcds;
  return want < res ? want : res;
}

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_mfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = MDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<mfma_stage_kernel<N, STAGE, MAT, SRC>>(kThreads, ntiles);
  mfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, kThreads, 0, s>>>(
      static_cast<const float*>(a.u_in), static_cast<float*>(a.out), static_cast<float*>(a.res),
      static_cast<const float*>(a.geo), a.fcode, static_cast<const float*>(a.mat),
      static_cast<const float*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? float(a.a) : 0.f, STAGE ? float(a.b) : 0.f, STAGE ? float(a.dt) : 0.f, a.src);
  return hipGetLastError();
}

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_hmfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = HDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<hmfma_stage_kernel<N, STAGE, MAT, SRC>>(HDims<N>::THREADS, ntiles);
  hmfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, HDims<N>::THREADS, 0, s>>>(
      static_cast<const float*>(a.u_in), static_cast<float*>(a.out), static_cast<float*>(a.res),
      static_cast<const float*>(a.geo), a.fcode, static_cast<const float*>(a.mat),
      static_cast<const float*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? float(a.a) : 0.f, STAGE ? float(a.b) : 0.f, STAGE ? float(a.dt) : 0.f, a.src);
  return hipGetLastError();
}

// The template variant for the stage mode, the medium and the scattered-field form.
template <int N, template <int, bool, bool, bool> class L>
hipError_t launch_variant(bool stage, const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const bool mat = a.mat != nullptr, src = a.src.rec != nullptr;
  if (stage) {
    if (mat) return src ? L<N, true, true, true>::run(ops, a, s) : L<N, true, true, false>::run(ops, a, s);
    return src ? L<N, true, false, true>::run(ops, a, s) : L<N, true, false, false>::run(ops, a, s);
  }
  if (mat) return src ? L<N, false, true, true>::run(ops, a, s) : L<N, false, true, false>::run(ops, a, s);
  return src ? L<N, false, false, true>::run(ops, a, s) : L<N, false, false, false>::run(ops, a, s);
}

template <int N, bool STAGE, bool MAT, bool SRC>
struct MfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_mfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N, bool STAGE, bool MAT, bool SRC>
struct HmfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_hmfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_dmfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = DDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<dmfma_stage_kernel<N, STAGE, MAT, SRC>>(DDims<N>::THREADS, ntiles);
  dmfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, DDims<N>::THREADS, 0, s>>>(
      static_cast<const double*>(a.u_in), static_cast<double*>(a.out), static_cast<double*>(a.res),
      static_cast<const double*>(a.geo), a.fcode, static_cast<const double*>(a.mat),
      static_cast<const double*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? a.a : 0.0, STAGE ? a.b : 0.0, STAGE ? a.dt : 0.0, a.src);
  return hipGetLastError();
}

template <int N, bool STAGE, bool MAT, bool SRC>
struct DmfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_dmfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_wmfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = WDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<wmfma_stage_kernel<N, STAGE, MAT, SRC>>(WDims<N>::THREADS, ntiles);
  wmfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, WDims<N>::THREADS, 0, s>>>(
      static_cast<const double*>(a.u_in), static_cast<double*>(a.out), static_cast<double*>(a.res),
      static_cast<const double*>(a.geo), a.fcode, static_cast<const double*>(a.mat),
      static_cast<const double*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? a.a : 0.0, STAGE ? a.b : 0.0, STAGE ? a.dt : 0.0, a.src);
  return hipGetLastError();
}

template <int N, bool STAGE, bool MAT, bool SRC>
struct WmfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_wmfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_bmfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = BDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<bmfma_stage_kernel<N, STAGE, MAT, SRC>>(BDims<N>::THREADS, ntiles);
  bmfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, BDims<N>::THREADS, 0, s>>>(
      static_cast<const float*>(a.u_in), static_cast<float*>(a.out), static_cast<float*>(a.res),
      static_cast<const float*>(a.geo), a.fcode, static_cast<const float*>(a.mat),
      static_cast<const uint16_t*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? float(a.a) : 0.f, STAGE ? float(a.b) : 0.f, STAGE ? float(a.dt) : 0.f, a.src);
  return hipGetLastError();
}

template <int N, bool STAGE, bool MAT, bool SRC>
struct BmfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_bmfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N, bool STAGE, bool MAT, bool SRC>
hipError_t launch_smfma_v(const OpsView& ops, const StageArgs& a, hipStream_t s) {
  const int E = SDims<N>::E;
  const int ntiles = (a.K + E - 1) / E;
  const int nb = persistent_grid<smfma_stage_kernel<N, STAGE, MAT, SRC>>(SDims<N>::THREADS, ntiles);
  smfma_stage_kernel<N, STAGE, MAT, SRC><<<nb, SDims<N>::THREADS, 0, s>>>(
      static_cast<const float*>(a.u_in), static_cast<float*>(a.out), static_cast<float*>(a.res),
      static_cast<const float*>(a.geo), a.fcode, static_cast<const float*>(a.mat),
      static_cast<const float*>(ops.opfrag), ops.fmask, ops.nbrnode, a.K, ntiles,
      STAGE ? float(a.a) : 0.f, STAGE ? float(a.b) : 0.f, STAGE ? float(a.dt) : 0.f, a.src);
  return hipGetLastError();
}

template <int N, bool STAGE, bool MAT, bool SRC>
struct SmfmaLaunch {
  static hipError_t run(const OpsView& o, const StageArgs& a, hipStream_t s) {
    return launch_smfma_v<N, STAGE, MAT, SRC>(o, a, s);
  }
};

template <int N>
hipError_t launch_hmfma_t(bool stage, const OpsView& ops, const StageArgs& a, hipStream_t s) {
  return launch_variant<N, HmfmaLaunch>(stage, ops, a, s);
}

template <int N>
hipError_t launch_mfma_t(bool stage, const OpsView& ops, const StageArgs& a, hipStream_t s) {
  return launch_variant<N, MfmaLaunch>(stage, ops, a, s);
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
  auto* mt = static_cast<const T*>(a.mat);
  auto* dr = static_cast<const T*>(ops.Dr);
  auto* ds = static_cast<const T*>(ops.Ds);
  auto* dt = static_cast<const T*>(ops.Dt);
  auto* lf = static_cast<const T*>(ops.LIFT);
  if (stage)
    stage_kernel<T, N, true><<<nblocks, kThreads, 0, s>>>(u, o, r, g, a.fcode, mt, dr, ds, dt, lf, ops.fmask,
                                                         ops.nbrnode, a.K, ntiles, T(a.a), T(a.b), T(a.dt), a.src);
  else
    stage_kernel<T, N, false><<<nblocks, kThreads, 0, s>>>(u, o, r, g, a.fcode, mt, dr, ds, dt, lf, ops.fmask,
                                                          ops.nbrnode, a.K, ntiles, T(0), T(0), T(0), a.src);
  return hipGetLastError();
}

// Canonical [6][K][Np] <-> internal [K][6][S] in chunks of CE consecutive user elements: the
// chunk's six canonical field blocks (CE Np contiguous words each) are read or written
// coalesced, and each element's internal block (6 S contiguous words at its internal position
// pos_of[e]) is written or read whole; the transposition happens in LDS ([CE][6][S]). Np, S
// and CE are compile-time constants, so the index arithmetic has no runtime divisions, and
// each phase issues all of a thread's loads before its first use (R1 / R2 rounds unrolled),
// so a thread keeps up to 32 loads in flight. Index arithmetic in I (32-bit where the arrays
// fit).
template <typename T, int N>
struct PermDims {
  static constexpr int Np = Dims<N>::Np, S = kRowStride<T, N>, RS = 6 * S;
  static constexpr int CE0 = (32 * 1024) / int(RS * sizeof(T));
  static constexpr int CE = CE0 < 1 ? 1 : (CE0 > 64 ? 64 : CE0);   // LDS tile <= 32 KB
  static constexpr int BLK = CE * Np;
  static constexpr int R1 = (6 * BLK + kThreads - 1) / kThreads;   // canonical-side rounds
  static constexpr int R2 = (CE * RS + kThreads - 1) / kThreads;   // internal-side rounds
};

template <typename T, int N, typename I>
__global__ __launch_bounds__(kThreads) void to_internal_kernel(const T* __restrict__ canon,
                                                               T* __restrict__ internal,
                                                               const int32_t* __restrict__ pos_of, int K) {
  using D = PermDims<T, N>;
  constexpr int NP = D::Np, S = D::S, RS = D::RS, CE = D::CE, BLK = D::BLK, R1 = D::R1, R2 = D::R2;
  static_assert(CE <= kThreads, "one position per thread");
  __shared__ __align__(16) T tile[CE * RS];
  __shared__ int32_t pos_s[CE];
  const int tid = threadIdx.x;
  for (int e0 = blockIdx.x * CE; e0 < K; e0 += gridDim.x * CE) {
    const int ne = min(CE, K - e0);
    T v[R1];
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int q = tid + k * kThreads;
      const int c = q / BLK, r = q - c * BLK, j = r / NP;
      v[k] = (q < 6 * BLK && j < ne) ? canon[(I(c) * K + e0) * NP + r] : T(0);
    }
    // the chunk's internal positions, read after the field loads (in-order completion: their
    // wait covers those loads, which are needed next anyway) and kept in LDS, so that the
    // stores below do not wait on a global load each
    if (tid < ne) pos_s[tid] = pos_of[e0 + tid];
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int q = tid + k * kThreads;
      const int c = q / BLK, r = q - c * BLK, j = r / NP, n = r - j * NP;
      if (q < 6 * BLK) tile[j * RS + c * S + n] = v[k];
    }
    if constexpr (S > NP)
      for (int q = tid; q < 6 * CE * (S - NP); q += kThreads) {
        const int row = q / (S - NP);
        tile[row * S + NP + (q - row * (S - NP))] = T(0);
      }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R2; ++k) {
      const int q = tid + k * kThreads, j = q / RS;
      if (q < CE * RS && j < ne) internal[I(pos_s[j]) * RS + (q - j * RS)] = tile[q];
    }
    __syncthreads();
  }
}

template <typename T, int N, typename I>
__global__ __launch_bounds__(kThreads) void to_canonical_kernel(const T* __restrict__ internal,
                                                                T* __restrict__ canon,
                                                                const int32_t* __restrict__ pos_of, int K) {
  using D = PermDims<T, N>;
  constexpr int NP = D::Np, S = D::S, RS = D::RS, CE = D::CE, BLK = D::BLK, R1 = D::R1, R2 = D::R2;
  static_assert(CE <= kThreads, "one position per thread");
  __shared__ __align__(16) T tile[CE * RS];
  __shared__ int32_t pos_s[CE];
  const int tid = threadIdx.x;
  const int stride = gridDim.x * CE;
  // internal positions of the first chunk; those of the next one are loaded during each chunk
  int pn = 0;
  if (tid < CE && blockIdx.x * CE + tid < K) pn = pos_of[blockIdx.x * CE + tid];
  for (int e0 = blockIdx.x * CE; e0 < K; e0 += stride) {
    const int ne = min(CE, K - e0);
    if (tid < CE) pos_s[tid] = pn;
    __syncthreads();
    T v[R2];
#pragma unroll
    for (int k = 0; k < R2; ++k) {
      const int q = tid + k * kThreads, j = q / RS;
      v[k] = (q < CE * RS && j < ne) ? internal[I(pos_s[j]) * RS + (q - j * RS)] : T(0);
    }
    if (tid < CE && e0 + stride + tid < K) pn = pos_of[e0 + stride + tid];
#pragma unroll
    for (int k = 0; k < R2; ++k) {
      const int q = tid + k * kThreads;
      if (q < CE * RS) tile[q] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R1; ++k) {
      const int q = tid + k * kThreads;
      const int c = q / BLK, r = q - c * BLK, j = r / NP, n = r - j * NP;
      if (q < 6 * BLK && j < ne) canon[(I(c) * K + e0) * NP + r] = tile[j * RS + c * S + n];
    }
    __syncthreads();
  }
}

template <typename T, int N>
__global__ __launch_bounds__(kThreads) void energy_kernel(const T* __restrict__ u, const T* __restrict__ M,
                                                          const T* __restrict__ geo, const T* __restrict__ mat,
                                                          int K, double* __restrict__ partial) {
  constexpr int NP = Dims<N>::Np, NS = kRowStride<T, N>;
  __shared__ double red[kThreads];
  double acc = 0.0;
  const int e0 = blockIdx.x * kEnergyBlockElems;
  const int e1 = min(K, e0 + kEnergyBlockElems);
  for (int q = threadIdx.x; q < (e1 - e0) * NP; q += kThreads) {
    const int e = e0 + q / NP, i = q % NP;
    const T* ue = u + size_t(e) * 6 * NS;
    double s = 0.0;
    for (int c = 0; c < 6; ++c) {
      double mu = 0.0;
      for (int j = 0; j < NP; ++j) mu += double(M[i * NP + j]) * double(ue[c * NS + j]);
      // eps weights the E fields and mu the H fields in a medium
      const double w = mat ? double(mat[size_t(e) * dgh::kMatStride + (c < 3 ? 2 : 3)]) : 1.0;
      s += w * mu * double(ue[c * NS + i]);
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
hipError_t launch_energy_t(const void* u, const void* M, const void* geo, const void* mat, int K,
                           double* partial, hipStream_t s) {
  const int nb = (K + kEnergyBlockElems - 1) / kEnergyBlockElems;
  energy_kernel<T, N><<<nb, kThreads, 0, s>>>(static_cast<const T*>(u), static_cast<const T*>(M),
                                              static_cast<const T*>(geo), static_cast<const T*>(mat), K,
                                              partial);
  return hipGetLastError();
}

// Sum of n partial energies by one workgroup: strided per-thread sums, then a tree in LDS
// (a fixed order, so the result does not depend on timing).
__global__ __launch_bounds__(kThreads) void sum_kernel(const double* __restrict__ partial, int n,
                                                       double* __restrict__ out) {
  __shared__ double red[kThreads];
  double acc = 0.0;
  for (int q = threadIdx.x; q < n; q += kThreads) acc += partial[q];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// The step's start time in the incident record (one thread).
__global__ void clock_kernel(double* rec, double v, int add) {
  if (threadIdx.x == 0 && blockIdx.x == 0) rec[8] = add ? rec[8] + v : v;
}

// The VALU kernel reads rows of Np words; an order whose rows are padded is served by the
// contraction kernel only.
template <typename T, int N>
hipError_t valu_stage(bool stage, const OpsView& o, const StageArgs& a, hipStream_t s) {
  if constexpr (kRowStride<T, N> == Dims<N>::Np) return launch_stage_t<T, N>(stage, o, a, s);
  else return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_stage(int N, bool stage, const OpsView& o, const StageArgs& a, hipStream_t s) {
  switch (N) {
    case 1: return valu_stage<T, 1>(stage, o, a, s);
    case 2: return valu_stage<T, 2>(stage, o, a, s);
    case 3: return valu_stage<T, 3>(stage, o, a, s);
    case 4: return valu_stage<T, 4>(stage, o, a, s);
    case 5: return valu_stage<T, 5>(stage, o, a, s);
    case 6: return valu_stage<T, 6>(stage, o, a, s);
    case 7: return valu_stage<T, 7>(stage, o, a, s);
    case 8: return valu_stage<T, 8>(stage, o, a, s);
    case 9: return valu_stage<T, 9>(stage, o, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t dispatch_energy(int N, const void* u, const void* M, const void* geo, const void* mat, int K,
                           double* p, hipStream_t s) {
  switch (N) {
    case 1: return launch_energy_t<T, 1>(u, M, geo, mat, K, p, s);
    case 2: return launch_energy_t<T, 2>(u, M, geo, mat, K, p, s);
    case 3: return launch_energy_t<T, 3>(u, M, geo, mat, K, p, s);
    case 4: return launch_energy_t<T, 4>(u, M, geo, mat, K, p, s);
    case 5: return launch_energy_t<T, 5>(u, M, geo, mat, K, p, s);
    case 6: return launch_energy_t<T, 6>(u, M, geo, mat, K, p, s);
    case 7: return launch_energy_t<T, 7>(u, M, geo, mat, K, p, s);
    case 8: return launch_energy_t<T, 8>(u, M, geo, mat, K, p, s);
    case 9: return launch_energy_t<T, 9>(u, M, geo, mat, K, p, s);
  }
  return hipErrorInvalidValue;
}

int grid_for(int64_t total) {
  int64_t b = (total + kThreads - 1) / kThreads;
  return int(b < 65536 ? (b < 1 ? 1 : b) : 65536);
}

}  // namespace

int opcat_words(int N, bool f64) {
  if (f64 && N == 4) return WDims<4>::OPC;   // FP64 N = 4: three padded column tiles, no tail
  switch (N) {
    case 3: return MDims<3>::OPC;
    case 4: return MDims<4>::OPC;
    case 5: return HDims<5>::OPC;
    case 6: return HDims<6>::OPC;
    case 7: return HDims<7>::OPC;
  }
  return 0;
}

bool mfma_order(int N) { return contraction_order(N); }

bool dmfma_order(int N) { return N >= 3 && N <= 7; }

bool bf16x3_order(int N) { return N >= 5 && N <= 7; }

int bopcat_words(int N) {
  switch (N) {
    case 5: return BDims<5>::OPW;
    case 6: return BDims<6>::OPW;
    case 7: return BDims<7>::OPW;
  }
  return 0;
}

namespace {
template <typename D>
void bopfrag_source_t(int w, int* n, int* blk, int* col, int* part) {
  // w = ((nt KB + b) 64 + lane) 16 + part 8 + j: column 16 nt + lane mod 16 of the operator,
  // k = 32 b + 8 (lane / 16) + j of the concatenation [D_r | D_s | D_t | LIFT]
  const int j = w % 8, pt = (w / 8) % 2, lane = (w / 16) % 64, tb = w / 1024;
  const int b = tb % D::KB, nt = tb / D::KB;
  *n = 16 * nt + lane % 16;
  *part = pt;
  const int k = 32 * b + 8 * (lane / 16) + j;
  if (k < D::KV) {
    *blk = k / D::NP8;
    *col = k % D::NP8;
    if (*col >= D::Np) *col = D::Np;   // padding node: outside the operator (zero)
  } else {
    *blk = 3;
    *col = k - D::KV;                  // >= 4 Nfp in the padding: outside the operator (zero)
  }
}
}  // namespace

void bopfrag_source(int N, int w, int* n, int* blk, int* col, int* part) {
  switch (N) {
    case 5: return bopfrag_source_t<BDims<5>>(w, n, blk, col, part);
    case 6: return bopfrag_source_t<BDims<6>>(w, n, blk, col, part);
    case 7: return bopfrag_source_t<BDims<7>>(w, n, blk, col, part);
  }
  *n = *blk = *col = *part = -1;
}

int row_stride(int N, bool f64) {
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6;
  return (!f64 && contraction_order(N)) ? (Np + 3) / 4 * 4 : Np;
}

namespace {
// Decodes a column k of the padded concatenation [D_r | D_s | D_t] (NPP columns each) + LIFT
// (NF columns) into operator block and column within it.
template <typename D>
void opcat_column(int k, int* blk, int* col) {
  if (k < D::KV) {
    *blk = k / D::NPP;
    *col = k % D::NPP;
  } else {
    *blk = 3;
    *col = k - D::KV;
  }
}

template <typename D>
void opfrag_source_t(int w, int* n, int* blk, int* col) {
  const int per_tile = D::KS * 64;
  int k = 0;
  if (w < D::NT * per_tile) {
    const int nt = w / per_tile, r = w - nt * per_tile;
    if (r < D::NQ * 256) {   // quad q, lane, step s
      const int q = r / 256, lane = (r / 4) % 64, s = r % 4, g = lane / 16;
      *n = 16 * nt + lane % 16;
      if (q < D::QV) {
        const int jb = q / 3, mu = q % 3;
        k = mu * D::NPP + 16 * jb + 4 * g + s;
      } else {
        k = D::KV + 16 * (q - D::QV) + 4 * g + s;
      }
    } else {                 // single (r, mu), lane
      const int r1 = r - D::NQ * 256, sg = r1 / 64, lane = r1 % 64, g = lane / 16;
      const int rr = sg / 3, mu = sg % 3;
      *n = 16 * nt + lane % 16;
      k = mu * D::NPP + 16 * D::VB + 4 * rr + g;
    }
  } else {                   // tail: quads [q][g][c][s], then singles [(r, mu)][g][c]
    const int r = w - D::NT * per_tile;
    if (r < D::NQ * 64) {
      const int q = r / 64, g = (r / 16) % 4, c = (r / 4) % 4, s = r % 4;
      *n = 16 * D::NT + c;
      k = q < D::QV ? (q % 3) * D::NPP + 16 * (q / 3) + 4 * g + s : D::KV + 16 * (q - D::QV) + 4 * g + s;
    } else {
      const int r1 = r - D::NQ * 64, sg = r1 / 16, g = (r1 / 4) % 4, c = r1 % 4;
      *n = 16 * D::NT + c;
      k = (sg % 3) * D::NPP + 16 * D::VB + 4 * (sg / 3) + g;
    }
  }
  opcat_column<D>(k, blk, col);
}
}  // namespace

void opfrag_source(int N, bool f64, int w, int* n, int* blk, int* col) {
  if (f64 && N == 4) return opfrag_source_t<WDims<4>>(w, n, blk, col);
  switch (N) {
    case 3: return opfrag_source_t<MDims<3>>(w, n, blk, col);
    case 4: return opfrag_source_t<MDims<4>>(w, n, blk, col);
    case 5: return opfrag_source_t<HDims<5>>(w, n, blk, col);
    case 6: return opfrag_source_t<HDims<6>>(w, n, blk, col);
    case 7: return opfrag_source_t<HDims<7>>(w, n, blk, col);
  }
  *n = *blk = *col = -1;
}

hipError_t launch_stage(int N, bool f64, bool stage, const OpsView& ops, const StageArgs& a,
                        hipStream_t s) {
  if (a.split_bf16) {
    if (N == 5) return launch_variant<5, BmfmaLaunch>(stage, ops, a, s);
    if (N == 6) return launch_variant<6, BmfmaLaunch>(stage, ops, a, s);
    if (N == 7) return launch_variant<7, BmfmaLaunch>(stage, ops, a, s);
    return hipErrorInvalidValue;
  }
  if (f64 && ops.opfrag) {
    if (N == 3) return launch_variant<3, DmfmaLaunch>(stage, ops, a, s);
    if (N == 4) return launch_variant<4, WmfmaLaunch>(stage, ops, a, s);
    if (N == 5) return launch_variant<5, WmfmaLaunch>(stage, ops, a, s);
    if (N == 6) return launch_variant<6, WmfmaLaunch>(stage, ops, a, s);
    if (N == 7) return launch_variant<7, WmfmaLaunch>(stage, ops, a, s);
  }
  if (!f64 && ops.opfrag) {
    if (N == 3) return a.wide_tiles ? launch_mfma_t<3>(stage, ops, a, s) : launch_variant<3, SmfmaLaunch>(stage, ops, a, s);
    if (N == 4) return launch_mfma_t<4>(stage, ops, a, s);
    if (N == 5) return launch_hmfma_t<5>(stage, ops, a, s);
    if (N == 6) return launch_hmfma_t<6>(stage, ops, a, s);
    if (N == 7) return launch_hmfma_t<7>(stage, ops, a, s);
  }
  return f64 ? dispatch_stage<double>(N, stage, ops, a, s) : dispatch_stage<float>(N, stage, ops, a, s);
}

namespace {
template <typename T, int N, bool TO_INTERNAL>
hipError_t launch_permute_t(const void* from, void* to, const int32_t* pos_of, int K, hipStream_t s) {
  using D = PermDims<T, N>;
  if (K <= 0) return hipSuccess;
  const int64_t chunks = (int64_t(K) + D::CE - 1) / D::CE;
  const int g = int(chunks < 8192 ? chunks : 8192);
  const bool narrow = int64_t(K) * D::RS < INT32_MAX;
  auto* f = static_cast<const T*>(from);
  auto* t = static_cast<T*>(to);
  if (TO_INTERNAL) {
    if (narrow) to_internal_kernel<T, N, int32_t><<<g, kThreads, 0, s>>>(f, t, pos_of, K);
    else to_internal_kernel<T, N, int64_t><<<g, kThreads, 0, s>>>(f, t, pos_of, K);
  } else {
    if (narrow) to_canonical_kernel<T, N, int32_t><<<g, kThreads, 0, s>>>(f, t, pos_of, K);
    else to_canonical_kernel<T, N, int64_t><<<g, kThreads, 0, s>>>(f, t, pos_of, K);
  }
  return hipGetLastError();
}

template <typename T, bool TO_INTERNAL>
hipError_t launch_permute(int N, const void* from, void* to, const int32_t* pos_of, int K, hipStream_t s) {
  switch (N) {
    case 1: return launch_permute_t<T, 1, TO_INTERNAL>(from, to, pos_of, K, s);
    case 2: return launch_permute_t<T, 2, TO_INTERNAL>(from, to, pos_of, K, s);
    case 3: return launch_permute_t<T, 3, TO_INTERNAL>(from, to, pos_of, K, s);
    case 4: return launch_permute_t<T, 4, TO_INTERNAL>(from, to, pos_of, K, s);
    case 5: return launch_permute_t<T, 5, TO_INTERNAL>(from, to, pos_of, K, s);
    case 6: return launch_permute_t<T, 6, TO_INTERNAL>(from, to, pos_of, K, s);
    case 7: return launch_permute_t<T, 7, TO_INTERNAL>(from, to, pos_of, K, s);
    case 8: return launch_permute_t<T, 8, TO_INTERNAL>(from, to, pos_of, K, s);
    case 9: return launch_permute_t<T, 9, TO_INTERNAL>(from, to, pos_of, K, s);
  }
  return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_to_internal(int N, bool f64, const void* canon, void* internal, const int32_t* pos_of,
                              int K, hipStream_t s) {
  return f64 ? launch_permute<double, true>(N, canon, internal, pos_of, K, s)
             : launch_permute<float, true>(N, canon, internal, pos_of, K, s);
}

hipError_t launch_to_canonical(int N, bool f64, const void* internal, void* canon, const int32_t* pos_of,
                               int K, hipStream_t s) {
  return f64 ? launch_permute<double, false>(N, internal, canon, pos_of, K, s)
             : launch_permute<float, false>(N, internal, canon, pos_of, K, s);
}

hipError_t launch_energy(int N, bool f64, const void* u, const void* M, const void* geo, const void* mat,
                         int K, double* partial, hipStream_t s) {
  return f64 ? dispatch_energy<double>(N, u, M, geo, mat, K, partial, s)
             : dispatch_energy<float>(N, u, M, geo, mat, K, partial, s);
}

namespace {
__global__ __launch_bounds__(kThreads) void zero_kernel(uint4* __restrict__ p, size_t n16, uint8_t* __restrict__ tail,
                                                        int ntail) {
  const size_t stride = size_t(gridDim.x) * kThreads;
  for (size_t i = size_t(blockIdx.x) * kThreads + threadIdx.x; i < n16; i += stride) p[i] = uint4{0u, 0u, 0u, 0u};
  if (blockIdx.x == 0 && int(threadIdx.x) < ntail) tail[threadIdx.x] = 0;
}
}  // namespace

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 16) return hipErrorInvalidValue;
  const size_t n16 = bytes / 16;
  const int ntail = int(bytes % 16);
  const int g = grid_for(int64_t(n16 > 0 ? n16 : 1));
  zero_kernel<<<g, kThreads, 0, s>>>(static_cast<uint4*>(p), n16, static_cast<uint8_t*>(p) + n16 * 16, ntail);
  return hipGetLastError();
}

hipError_t launch_advance_clock(double* rec, double dt, hipStream_t s) {
  clock_kernel<<<1, 64, 0, s>>>(rec, dt, 1);
  return hipGetLastError();
}

hipError_t launch_set_clock(double* rec, double t, hipStream_t s) {
  clock_kernel<<<1, 64, 0, s>>>(rec, t, 0);
  return hipGetLastError();
}

hipError_t launch_sum(const double* partial, int n, double* out, hipStream_t s) {
  sum_kernel<<<1, kThreads, 0, s>>>(partial, n, out);
  return hipGetLastError();
}

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return e;
  if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  double* p = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
  if (cur != device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

double* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

}  // namespace dgk

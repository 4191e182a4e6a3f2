/*
 * dg.h — C ABI of libdg: nodal discontinuous Galerkin for Maxwell's equations on tetrahedra,
 * on one AMD Instinct MI355X (gfx950).
 *
 * The library evaluates the semi-discrete DG operator of the paper's Sec. 2
 * (eq. semidiscrete-dg: du/dt = -sum_nu D^nu F(u) + L[n.F - (n.F)*]) for Maxwell's equations
 * (Sec. 6, eq. maxwells-claws) in vacuum or in a medium with piecewise-constant eps and mu,
 * with the impedance-weighted upwind flux of Sec. 6, perfectly conducting walls (mirror state
 * E+ = -E-, H+ = H-) and absorbing faces (zero exterior state, the characteristic absorbing
 * condition named for the scattering example of Sec. 6), and advances it with the five-stage
 * fourth-order low-storage Runge-Kutta method named in Sec. 6.
 *
 * Conventions
 *   Fields: six components in the order Ex, Ey, Ez, Hx, Hy, Hz.
 *   Canonical field layout: [6][K][Np] contiguous, user element order, reference node order
 *   (node lattice (i,j,k), i+j+k <= N, k outermost, then j, i innermost), after the
 *   orientation fix below. Values are in the handle's working precision (double for DG_F64,
 *   float for DG_F32).
 *   Orientation fix: an element with det[v2-v1, v3-v1, v4-v1] < 0 has its local vertices 3
 *   and 4 (1-based) swapped before anything else; node order refers to the fixed element.
 *   Reference faces: F1 = (v1,v2,v3), F2 = (v1,v2,v4), F3 = (v2,v3,v4), F4 = (v1,v3,v4);
 *   face nodes of each face in ascending node index.
 *   Streams: every call that takes `stream` (a hipStream_t, NULL = the null stream) enqueues
 *   its device work there and does not synchronise, unless stated otherwise.
 *   Errors: every function returns 0 on success or a negative DG_E_* code; the text of the
 *   last error of the calling thread is returned by dg_last_error(). No function aborts.
 *   Thread safety: a handle must not be used by two threads at once.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DG_OK 0
#define DG_E_ARG (-1)         /* invalid argument (NULL pointer, bad size, bad option) */
#define DG_E_MESH (-2)        /* invalid mesh: degenerate element, face shared by > 2 elements */
#define DG_E_UNSUPPORTED (-3) /* order outside 1..9, unknown precision, DG_BF16X3 outside 5..7 */
#define DG_E_OOM (-4)         /* device allocation failed or the workspace is too small */
#define DG_E_HIP (-5)         /* a HIP runtime call failed; message in dg_last_error() */
#define DG_E_STATE (-6)       /* handle has no device state (built with device = -1) */
#define DG_E_NUMERIC (-7)     /* dg_solve's numeric monitor found a non-finite or growing energy */

typedef struct dg_handle dg_handle;

/* Working precision. DG_BF16X3 (orders 5..7): FP32 state, fluxes and RK update; the volume
 * and lift contraction splits each operand and operator value x into x_hi + x_lo (bf16 each)
 * and takes x_hi y_hi + x_hi y_lo + x_lo y_hi on the bf16 matrix cores with FP32 accumulation
 * (about 3 * 2^-18 relative error per product); field arrays are float. */
typedef enum { DG_F64 = 0, DG_F32 = 1, DG_BF16X3 = 2 } dg_precision;

/* Mesh description. All arrays are host memory owned by the caller and only read during
 * the call that receives them. */
typedef struct {
  int32_t nverts;         /* number of vertices */
  const double* vxyz;     /* nverts x 3, row-major coordinates */
  int32_t K;              /* number of tetrahedra, 1 <= K < 2^26 */
  const int32_t* etov;    /* K x 4 vertex ids, 0-based, any orientation */
  const int8_t* face_bc;  /* K x 4 or NULL, face f of element k being the triple F(f+1) of
                             etov[k] as given (before the orientation fix): 0 = automatic
                             (an unmatched face is a perfectly conducting wall), 1 = wall,
                             2 = absorbing, 3 = scatterer (scattered-field form, see
                             dg_set_incident); nonzero on a matched face is DG_E_MESH */
  const double* eps;      /* K permittivities (> 0, finite) or NULL (= 1 everywhere) */
  const double* mu;       /* K permeabilities (> 0, finite) or NULL (= 1 everywhere);
                             a bad value is DG_E_ARG */
} dg_mesh;

typedef struct {
  int32_t order;     /* polynomial order N, 1..9 (matrix-core kernels at 3..7) */
  int32_t precision; /* dg_precision */
  int32_t reorder;   /* 0 = keep user element order internally, 1 = Morton locality order */
  int32_t device;    /* HIP device ordinal, or -1 for a host-only handle (builder outputs
                        only: dg_info, dg_nodes, dg_get_maps, dg_get_operators) */
  int32_t checks;    /* numeric monitor of dg_solve: 0 = off; M > 0 = after every M steps the
                        energy must be finite and (without scatterer faces) not above its value
                        at the start of the call by more than 1e-10 (FP64) or 1e-4 (otherwise),
                        else dg_solve stops with DG_E_NUMERIC; each check synchronises `stream` */
  int32_t tile_id;   /* stage kernel: 0 = the library's default (the contraction kernel where
                        the order and precision have one), 1 = element-wise kernel (one thread
                        per element node; not FP32 N = 4, whose rows are padded, nor DG_BF16X3),
                        2 = contraction kernel (FP32 and FP64 N = 3..7, DG_BF16X3),
                        3 = contraction kernel with 16-element tiles instead of 8 (FP32 N = 3);
                        DG_E_UNSUPPORTED otherwise. An autotuner picks it per order, precision
                        and mesh size (paper_0901_1024_amd.tune) */
  int32_t reserved[2];
} dg_opts;

/* Sizes of a handle. */
typedef struct {
  int32_t order, Np, Nfp, K, precision, device;
  int64_t state_words;     /* 6 * K * Np: length of one canonical field array */
  size_t workspace_bytes;  /* device memory the handle uses */
} dg_info_t;

/* Device memory the handle needs for this mesh and options, in bytes (host-only work:
 * builds nothing on the device). */
int dg_setup_query(const dg_mesh* mesh, const dg_opts* opts, size_t* workspace_bytes);

/* Build the reference operators (Sec. 2, eqs. dg-global-matrices, dg-reference-matrices,
 * Fig. lifting-matrix), connectivity, geometric factors and face records in FP64 on the
 * host, then upload them. `dev_workspace` is device memory of at least `workspace_bytes`
 * (from dg_setup_query) owned by the caller and kept alive until dg_free, or NULL to let
 * the library allocate. The uploads are enqueued on `stream`; the call returns after they
 * complete. Fields start at zero. On failure *out is set to NULL. */
int dg_setup(const dg_mesh* mesh, const dg_opts* opts, void* dev_workspace,
             size_t workspace_bytes, void* stream, dg_handle** out);

/* Release the handle (and the device memory the library allocated). NULL is accepted. */
int dg_free(dg_handle* h);

/* Text of the last error on this thread ("" if none). */
const char* dg_last_error(void);

int dg_info(const dg_handle* h, dg_info_t* info);

/* Physical node coordinates, host array 3 x K x Np (x, then y, then z; canonical order). */
int dg_nodes(const dg_handle* h, double* xyz);

/* Canonical face-node maps, host arrays K x 4 x Nfp of flat node ids k*Np + n: vmapM is the
 * node of face f of element k, vmapP the coinciding node of the neighbour across that face
 * (itself on a wall). */
int dg_get_maps(const dg_handle* h, int32_t* vmapM, int32_t* vmapP);

/* Reference operators in FP64, host arrays: Dr, Ds, Dt (Np x Np row-major), LIFT
 * (Np x 4Nfp row-major), mass M (Np x Np), nodes rst (Np x 3). Any pointer may be NULL. */
int dg_get_operators(const dg_handle* h, double* Dr, double* Ds, double* Dt, double* LIFT,
                     double* M, double* rst);

/* Copy a canonical field array into the handle's state u (and zero the RK residual).
 * `u` is host memory if on_device == 0 (the call then synchronises `stream`), else device
 * memory. */
int dg_set_fields(dg_handle* h, const void* u, int on_device, void* stream);

/* Copy the handle's state u out as a canonical field array (host if on_device == 0, in
 * which case the call synchronises `stream`). */
int dg_get_fields(const dg_handle* h, void* u, int on_device, void* stream);

/* Semi-discrete right-hand side (Sec. 2, eq. semidiscrete-dg; Maxwell flux of Sec. 6):
 * rhs = curl/volume term + LIFT (Fscale * upwind flux), for the canonical device array
 * `u_dev`, written to the canonical device array `rhs_dev` (both 6*K*Np values of the
 * working precision, distinct buffers). Does not touch the handle's state. */
int dg_rhs(dg_handle* h, const void* u_dev, void* rhs_dev, void* stream);

/* One step of the five-stage low-storage RK4 method (Sec. 6) of size dt on the handle's
 * state: for each stage i, res = a_i res + dt rhs(u); u = u + b_i res. */
int dg_rk_step(dg_handle* h, double dt, void* stream);

/* nsteps calls of dg_rk_step, launched from a captured HIP graph of two steps. With
 * opts.checks = M > 0 the steps run in chunks of M, each followed by the energy check described
 * at dg_opts (DG_E_NUMERIC: the state holds the steps taken so far, dg_get_time tells when). */
int dg_solve(dg_handle* h, double dt, int64_t nsteps, void* stream);

/* Discrete energy 1/2 sum_k J_k (eps_k E_k^T M E_k + mu_k H_k^T M H_k) of the state (each
 * field component separately; eps = mu = 1 in vacuum), accumulated in double.
 * Synchronises `stream`. */
int dg_energy(const dg_handle* h, double* energy, void* stream);

/* ---- Scattered-field form (the incident-field formulation of the scattering example of
 * Sec. 6). The state is the scattered field; the total field is it plus a known incident plane
 * wave in vacuum, E_inc = p f(k.x - t), H_inc = (k x p) f(k.x - t), with profile
 * f(s) = c0 + c1 s + c2 sin(c3 s + c4). On scatterer faces (face_bc = 3) the total field meets
 * a perfectly conducting wall: E+ = -E- - 2 E_inc(x, t), H+ = H-. The operator then depends on
 * time: the handle keeps the time of its next step (initially 0; each RK step advances it by
 * dt, also inside dg_solve's graph), dg_rhs evaluates at that time and the RK stages at
 * t + c_i dt. Not available in a batch handle (DG_E_UNSUPPORTED at setup). */

/* Incident wave: direction k (3, normalised by the call), polarisation p (3, orthogonal to k;
 * its length is the amplitude) and profile (c0..c4). Computes k.x at every scatterer face node
 * in FP64 on the host and uploads it with the record; synchronises `stream`. Without this call
 * the incident field is zero and scatterer faces act as walls. DG_E_ARG if the mesh has no
 * scatterer faces or the arguments are not finite or p is not orthogonal to k. */
int dg_set_incident(dg_handle* h, const double* k, const double* p, const double* profile, void* stream);

/* Set the time of the handle's next step (any handle; it matters only with scatterer faces). */
int dg_set_time(dg_handle* h, double t, void* stream);

/* The time of the handle's next step (host-side copy; does not synchronise). */
int dg_get_time(const dg_handle* h, double* t);

/* The energy of dg_energy, computed without allocating anything and without synchronising:
 * for callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). The result (one double) is written to the device
 * pointer `energy_dev` on `stream`. The per-block partial sums go to a static device array of
 * the library (512 KiB on each device, set up by dg_setup), so K is limited to 4,194,304
 * elements (larger: DG_E_ARG, use dg_energy). Every call on a device shares that array: calls
 * that overlap on one device (other streams, other threads) race and must be ordered by the
 * caller. Nothing in the array needs to start at zero (each call writes every partial it
 * reads). The summation order differs from dg_energy's (tree against sequential), so the two
 * agree to rounding. */
int dg_energy_noalloc(const dg_handle* h, double* energy_dev, void* stream);

/* Time-step bound used by the tests and the benchmark: cfl * min over faces of 1/Fscale,
 * divided by N^2 (host-only). It assumes wave speed at most 1, i.e. eps * mu >= 1. */
int dg_stable_dt(const dg_handle* h, double cfl, double* dt);

/* ---- Batched form: many meshes of one order and precision in one handle -------------------
 * The meshes are concatenated (canonical elements of mesh i are [first[i], first[i+1]) of the
 * handle's canonical arrays); the locality order keeps each mesh contiguous, so one launch per
 * RK stage advances all of them, and dg_solve replays them from one captured graph. Each mesh
 * may have its own time step (dg_set_batch_dt): the right-hand side is linear in the
 * per-element inverse-map derivatives, Fscale and flux weights, so the RK stages read a copy
 * of those records scaled by the mesh's step and the dt argument of dg_rk_step / dg_solve
 * multiplies the per-mesh steps (pass 1.0). dg_rhs, dg_energy and the field calls see the
 * unscaled operator. Meshes may differ in K, geometry, face conditions and materials. */

/* Workspace bytes for dg_setup_batch with the same arguments. A batch handle holds a second
 * copy of the geometric records (and, in a medium, of the material records) scaled by each
 * mesh's time step, so its metadata takes twice the bytes of a plain handle's (26 words per
 * element, plus 20 in a medium, in the working precision). */
int dg_setup_query_batch(const dg_mesh* meshes, int32_t count, const dg_opts* opts,
                         size_t* workspace_bytes);

/* Like dg_setup for `count` meshes (count >= 1, total K < 2^26). */
int dg_setup_batch(const dg_mesh* meshes, int32_t count, const dg_opts* opts, void* dev_workspace,
                   size_t workspace_bytes, void* stream, dg_handle** out);

/* Number of meshes (1 for a plain handle) and, if `first` is not NULL, the count + 1 canonical
 * element offsets (host array). */
int dg_batch_info(const dg_handle* h, int32_t* count, int32_t* first);

/* dg_stable_dt of every mesh of the handle, `dt` holds count values (host-only). */
int dg_batch_stable_dt(const dg_handle* h, double cfl, double* dt);

/* Per-mesh time steps (count finite positive values, host array) for the RK stages of a batch
 * handle; the default is 1. Uploads the scaled records and synchronises `stream`. */
int dg_set_batch_dt(dg_handle* h, const double* dt, void* stream);

/* ---- Group: handles of any orders and precisions advanced together ----------------------
 * dg_group_solve advances every member handle by nsteps steps of its own dt (dt[i]; for a
 * batch member, the multiplier of its per-mesh steps) from one captured HIP graph: each
 * member's two-step sequence is a branch forked from and joined into the calling stream, with
 * no dependency between branches, so the device may run the members concurrently. Members
 * keep their own state, face conditions, clocks and ping-pong buffers; a member must not be
 * used elsewhere while the group solves, and must outlive the group. The numeric monitor of
 * dg_opts.checks does not run inside a group solve. */
typedef struct dg_group dg_group;

/* count >= 1 distinct device handles on one device. */
int dg_group_create(dg_handle* const* members, int32_t count, dg_group** out);

int dg_group_free(dg_group* g);

/* dt: count finite time steps (host array). */
int dg_group_solve(dg_group* g, const double* dt, int64_t nsteps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */

// C ABI of libdg (see include/dg.h): handle lifetime, host build, uploads, and the stage
// sequence of the five-stage low-storage RK4 method of Sec. 6.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "dg.h"
#include "host/meshbuild.hpp"
#include "host/refops.hpp"
#include "kernels.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Carpenter-Kennedy five-stage fourth-order 2N-storage coefficients.
constexpr double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                            -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
constexpr double kRkB[5] = {1432997174477.0 / 9575080441755.0, 5161836677717.0 / 13612068292357.0,
                            1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                            2277821191437.0 / 14882151754819.0};
// stage times: stage i evaluates the operator at t + c_i dt
constexpr double kRkC[5] = {0.0, 1432997174477.0 / 9575080441755.0, 2526269341429.0 / 6820363962896.0,
                            2006345519317.0 / 3224310063776.0, 2802321613138.0 / 2924317926251.0};

struct Layout {
  size_t state = 0;   // bytes of one canonical [6][K][Np] array
  size_t istate = 0;  // bytes of one internal [K][6][S] array (S = dgk::row_stride)
  size_t off_u0, off_u1, off_res, off_tmp, off_geo, off_fcode, off_ops, off_fmask, off_nbr,
      off_pos_of, off_partial, off_opcat, off_mat, off_geo_dt, off_mat_dt, off_src,
      off_phase, total;
  size_t opcat_bytes = 0, mat_bytes = 0, geo_dt_bytes = 0, mat_dt_bytes = 0, src_bytes = 0, phase_bytes = 0;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Bytes of the fragment-ordered concatenated operator of the contraction kernels: FP32, FP64
// where an FP64 contraction kernel serves the order (same word order in both precisions), or
// the split-BF16 table (16-bit words).
bool contraction_kernel(int N, int prec) {
  return prec == DG_BF16X3 ? dgk::bf16x3_order(N) : prec == DG_F32 ? dgk::mfma_order(N) : dgk::dmfma_order(N);
}

// tile_id 0 resolved: the contraction kernel where there is one
int resolve_tile(int N, int prec, int tile_id) {
  return tile_id ? tile_id : (contraction_kernel(N, prec) ? 2 : 1);
}

size_t opfrag_bytes_for(int N, int prec, int tile_id = 0) {
  if (resolve_tile(N, prec, tile_id) < 2) return 0;
  if (prec == DG_BF16X3) return size_t(dgk::bopcat_words(N)) * 2;
  const bool used = prec == DG_F32 ? dgk::mfma_order(N) : dgk::dmfma_order(N);
  return used ? size_t(dgk::opcat_words(N, prec == DG_F64)) * (prec == DG_F64 ? 8 : 4) : 0;
}

// Nearest bf16 value (round to nearest even) of a double, as a double; its bit pattern is
// that of the float of the same value, shifted right by 16.
double round_bf16(double x) {
  if (x == 0.0 || !std::isfinite(x)) return x;
  int e = 0;
  const double f = std::frexp(x, &e);   // x = f 2^e, 0.5 <= |f| < 1: 8 significant bits
  return std::ldexp(std::nearbyint(std::ldexp(f, 8)), e - 8);
}

uint16_t bf16_bits(double v) {   // v is a bf16 value
  const float f = static_cast<float>(v);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return static_cast<uint16_t>(u >> 16);
}

// batch: a second copy of the geometric (and material) records scaled by each mesh's time
// step, read by the RK stages (the right-hand side is linear in them).
// nscat: scatterer faces (scattered-field form): an incident record and Nfp phases per face,
// always in double.
Layout make_layout(int K, int N, int Np, int Nfp, int prec, bool material, bool batch = false,
                   int64_t nscat = 0, int tile_id = 0) {
  const size_t ts = prec == DG_F64 ? 8 : 4;
  Layout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o += align256(bytes);
    return at;
  };
  L.state = size_t(K) * 6 * Np * ts;
  L.istate = size_t(K) * 6 * dgk::row_stride(N, ts == 8) * ts;
  L.off_u0 = take(L.istate);
  L.off_u1 = take(L.istate);
  L.off_res = take(L.istate);
  L.off_tmp = take(L.istate);   // an internal array, or a canonical one (state <= istate)
  L.off_geo = take(size_t(K) * dgh::kGeoStride * ts);
  L.off_fcode = take(size_t(K) * 4 * sizeof(int32_t));
  L.off_ops = take((size_t(4) * Np * Np + size_t(Np) * 4 * Nfp) * ts);
  L.off_fmask = take(size_t(4) * Nfp * sizeof(int32_t));
  L.off_nbr = take(size_t(96) * Nfp * sizeof(int32_t));
  L.off_pos_of = take(size_t(K) * sizeof(int32_t));
  L.off_partial = take(size_t((K + dgk::kEnergyBlockElems - 1) / dgk::kEnergyBlockElems) * sizeof(double));
  L.opcat_bytes = opfrag_bytes_for(N, prec, tile_id);
  L.off_opcat = take(L.opcat_bytes);
  L.mat_bytes = material ? size_t(K) * dgh::kMatStride * ts : 0;
  L.off_mat = take(L.mat_bytes);
  L.geo_dt_bytes = batch ? size_t(K) * dgh::kGeoStride * ts : 0;
  L.off_geo_dt = take(L.geo_dt_bytes);
  L.mat_dt_bytes = batch ? L.mat_bytes : 0;
  L.off_mat_dt = take(L.mat_dt_bytes);
  L.src_bytes = nscat ? size_t(dgk::kSrcRecWords) * sizeof(double) : 0;
  L.off_src = take(L.src_bytes);
  L.phase_bytes = size_t(nscat) * Nfp * sizeof(double);
  L.off_phase = take(L.phase_bytes);
  L.total = o;
  return L;
}

// Scatterer faces requested by face_bc (value 3).
int64_t count_scatterers(const dg_mesh* mesh) {
  int64_t n = 0;
  if (mesh && mesh->face_bc)
    for (int64_t q = 0; q < int64_t(mesh->K) * 4; ++q) n += mesh->face_bc[q] == 3;
  return n;
}

int check_inputs(const dg_mesh* mesh, const dg_opts* opts) {
  if (!mesh || !opts) return fail(DG_E_ARG, "mesh and opts must not be NULL");
  if (!mesh->vxyz || !mesh->etov) return fail(DG_E_ARG, "vxyz and etov must not be NULL");
  if (mesh->K <= 0 || mesh->nverts < 4) return fail(DG_E_ARG, "empty mesh");
  if (opts->order < 1 || opts->order > 9) return fail(DG_E_UNSUPPORTED, "order must be in 1..9");
  if (opts->precision != DG_F64 && opts->precision != DG_F32 && opts->precision != DG_BF16X3)
    return fail(DG_E_UNSUPPORTED, "unknown precision");
  if (opts->precision == DG_BF16X3 && !dgk::bf16x3_order(opts->order))
    return fail(DG_E_UNSUPPORTED, "the split-BF16 contraction serves orders 5..7");
  if (opts->reorder < 0 || opts->reorder > 1) return fail(DG_E_ARG, "reorder must be 0 or 1");
  if (opts->checks < 0) return fail(DG_E_ARG, "checks must be >= 0");
  if (opts->tile_id < 0 || opts->tile_id > 3) return fail(DG_E_ARG, "tile_id must be 0, 1, 2 or 3");
  if (opts->tile_id == 3 && !(opts->precision == DG_F32 && opts->order == 3))
    return fail(DG_E_UNSUPPORTED, "16-element contraction tiles serve FP32 N = 3 only");
  if (opts->tile_id == 2 && !contraction_kernel(opts->order, opts->precision))
    return fail(DG_E_UNSUPPORTED, "no contraction kernel for this order and precision");
  if (opts->tile_id == 1 && (opts->precision == DG_BF16X3 ||
                             (opts->precision == DG_F32 && dgk::row_stride(opts->order, false) !=
                                                               (opts->order + 1) * (opts->order + 2) * (opts->order + 3) / 6)))
    return fail(DG_E_UNSUPPORTED, "no element-wise kernel for this order and precision");
  return DG_OK;
}

}  // namespace

struct dg_handle {
  dgh::RefOps ref;
  dgh::MeshData mesh;
  std::vector<double> mat;   // material records (internal order); empty in vacuum
  // batch of meshes: canonical element ranges [mesh_first[i], mesh_first[i+1]), the mesh of
  // each user element, and the unscaled geometric records in internal order
  bool batch = false;
  std::vector<int32_t> mesh_first, mesh_of;
  std::vector<double> geo_int;
  int N = 0, Np = 0, S = 0, Nfp = 0, K = 0, prec = 0, device = -1;
  size_t ts = 8;
  Layout lay;
  char* ws = nullptr;
  bool own_ws = false;
  int cur = 0;
  hipStream_t cap_stream = nullptr;
  // captured two-step graphs, one per parity of the ping-pong state (h->cur at capture), so
  // that a solve after an odd number of steps replays rather than re-captures
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  hipGraph_t graph[2] = {nullptr, nullptr};
  double graph_dt[2] = {0.0, 0.0};
  // scattered-field form: number of scatterer faces and the time at the start of the next
  // step (the device keeps the same value in the incident record; both add dt per step)
  int64_t nscat = 0;
  double t = 0.0;
  int checks = 0;   // numeric monitor interval of dg_solve (0: off)
  int tile = 0;     // stage kernel family (dg_opts.tile_id, 0 resolved)

  bool f64() const { return prec == DG_F64; }
  void* at(size_t off) const { return ws + off; }
  void* u(int i) const { return at(i == 0 ? lay.off_u0 : lay.off_u1); }
  dgk::OpsView ops() const {
    const size_t nn = size_t(Np) * Np * ts;
    dgk::OpsView o;
    o.Dr = at(lay.off_ops);
    o.Ds = at(lay.off_ops + nn);
    o.Dt = at(lay.off_ops + 2 * nn);
    o.M = at(lay.off_ops + 3 * nn);
    o.LIFT = at(lay.off_ops + 4 * nn);
    o.fmask = static_cast<const int32_t*>(at(lay.off_fmask));
    o.nbrnode = static_cast<const int32_t*>(at(lay.off_nbr));
    o.opfrag = lay.opcat_bytes ? at(lay.off_opcat) : nullptr;
    return o;
  }
  void drop_graph(int p) {
    if (gexec[p]) (void)hipGraphExecDestroy(gexec[p]);
    if (graph[p]) (void)hipGraphDestroy(graph[p]);
    gexec[p] = nullptr;
    graph[p] = nullptr;
  }
  void drop_graphs() {
    drop_graph(0);
    drop_graph(1);
  }
};

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(DG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                 \
  do {                                                \
    hipError_t _e = (call);                           \
    if (_e != hipSuccess) return hip_fail(_e, #call); \
  } while (0)

template <typename T>
std::vector<char> convert(const std::vector<double>& v) {
  std::vector<char> out(v.size() * sizeof(T));
  T* p = reinterpret_cast<T*>(out.data());
  for (size_t i = 0; i < v.size(); ++i) p[i] = static_cast<T>(v[i]);
  return out;
}

std::vector<char> to_prec(const std::vector<double>& v, bool f64) {
  return f64 ? convert<double>(v) : convert<float>(v);
}

int upload(dg_handle* h, hipStream_t s) {
  const auto& R = h->ref;
  const auto& M = h->mesh;
  const int K = h->K;
  // geometric records in internal order
  std::vector<double> geo(size_t(K) * dgh::kGeoStride);
  for (int i = 0; i < K; ++i)
    std::memcpy(&geo[size_t(i) * dgh::kGeoStride], &M.geo[size_t(M.elem_of[i]) * dgh::kGeoStride],
                sizeof(double) * dgh::kGeoStride);
  std::vector<double> ops;
  ops.reserve(size_t(4) * h->Np * h->Np + size_t(h->Np) * 4 * h->Nfp);
  for (const auto* m : {&R.Dr, &R.Ds, &R.Dt, &R.M}) ops.insert(ops.end(), m->begin(), m->end());
  ops.insert(ops.end(), R.LIFT.begin(), R.LIFT.end());
  std::vector<char> geo_b = to_prec(geo, h->f64()), ops_b = to_prec(ops, h->f64());
  if (h->lay.opcat_bytes && h->prec == DG_BF16X3) {
    // [Dr | Ds | Dt | LIFT] split once in FP64: hi = bf16(x), lo = bf16(x - hi)
    const int Np = h->Np, Nf4 = 4 * h->Nfp;
    std::vector<uint16_t> ob(size_t(dgk::bopcat_words(h->N)), 0);
    for (size_t w = 0; w < ob.size(); ++w) {
      int n = -1, blk = -1, col = -1, part = -1;
      dgk::bopfrag_source(h->N, int(w), &n, &blk, &col, &part);
      if (n < 0 || blk < 0 || blk > 3 || col < 0 || part < 0) return fail(DG_E_ARG, "internal: bad operator map");
      double x = 0.0;
      if (n < Np && blk < 3 && col < Np) {
        const std::vector<double>& Dm = blk == 0 ? R.Dr : blk == 1 ? R.Ds : R.Dt;
        x = Dm[size_t(n) * Np + col];
      } else if (n < Np && blk == 3 && col < Nf4) {
        x = R.LIFT[size_t(n) * Nf4 + col];
      }
      const double hi = round_bf16(x);
      ob[w] = bf16_bits(part == 0 ? hi : round_bf16(x - hi));
    }
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_opcat), ob.data(), ob.size() * 2, hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  } else if (h->lay.opcat_bytes) {
    // OpCat = [Dr | Ds | Dt | LIFT] in the lane order of the contraction kernel
    const int Np = h->Np, Nf4 = 4 * h->Nfp;
    std::vector<double> oc(size_t(dgk::opcat_words(h->N, h->f64())), 0.0);
    for (size_t w = 0; w < oc.size(); ++w) {
      int n = -1, blk = -1, col = -1;
      dgk::opfrag_source(h->N, h->f64(), int(w), &n, &blk, &col);
      if (n < 0 || blk < 0 || blk > 3 || col < 0) return fail(DG_E_ARG, "internal: bad operator fragment map");
      if (n >= Np) continue;
      if (blk < 3 && col < Np) {
        const std::vector<double>& Dm = blk == 0 ? R.Dr : blk == 1 ? R.Ds : R.Dt;
        oc[w] = Dm[size_t(n) * Np + col];
      } else if (blk == 3 && col < Nf4) {
        oc[w] = R.LIFT[size_t(n) * Nf4 + col];
      }
    }
    std::vector<char> oc_b = to_prec(oc, h->f64());
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_opcat), oc_b.data(), oc_b.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_geo), geo_b.data(), geo_b.size(), hipMemcpyHostToDevice, s));
  std::vector<char> mat_b;
  if (h->lay.mat_bytes) {
    mat_b = to_prec(h->mat, h->f64());
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_mat), mat_b.data(), mat_b.size(), hipMemcpyHostToDevice, s));
  }
  if (h->batch) {   // time-step-scaled copies start at dt = 1
    h->geo_int = geo;
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_geo_dt), geo_b.data(), geo_b.size(), hipMemcpyHostToDevice, s));
    if (h->lay.mat_dt_bytes)
      HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_mat_dt), mat_b.data(), mat_b.size(), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_ops), ops_b.data(), ops_b.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_fcode), M.face_code.data(), M.face_code.size() * 4,
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_fmask), R.Fmask.data(), R.Fmask.size() * 4, hipMemcpyHostToDevice, s));
  std::vector<int32_t> nbr(R.nbr_node.begin(), R.nbr_node.end());
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_nbr), nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_pos_of), M.pos_of.data(), size_t(K) * 4, hipMemcpyHostToDevice, s));
  if (h->nscat) {   // no incident wave until dg_set_incident: scatterer faces act as walls
    HIP_TRY(hipMemsetAsync(h->at(h->lay.off_src), 0, h->lay.src_bytes, s));
    HIP_TRY(hipMemsetAsync(h->at(h->lay.off_phase), 0, h->lay.phase_bytes, s));
  }
  HIP_TRY(hipMemsetAsync(h->u(0), 0, h->lay.istate, s));
  HIP_TRY(hipMemsetAsync(h->u(1), 0, h->lay.istate, s));
  HIP_TRY(hipMemsetAsync(h->at(h->lay.off_res), 0, h->lay.istate, s));
  HIP_TRY(hipStreamSynchronize(s));  // host staging buffers die at return
  return DG_OK;
}

int need_device(const dg_handle* h) {
  if (!h) return fail(DG_E_ARG, "NULL handle");
  if (h->device < 0) return fail(DG_E_STATE, "handle was built host-only (device = -1)");
  return DG_OK;
}

int set_device(const dg_handle* h) {
  HIP_TRY(hipSetDevice(h->device));
  return DG_OK;
}

int stage_launch(dg_handle* h, bool stage, const void* in, void* out, double a, double b, double dt,
                 hipStream_t s, double toff = 0.0) {
  dgk::StageArgs args;
  args.u_in = in;
  args.out = out;
  args.res = h->at(h->lay.off_res);
  const bool scaled = stage && h->batch;   // RK stages of a batch: per-mesh dt in the records
  args.geo = h->at(scaled ? h->lay.off_geo_dt : h->lay.off_geo);
  args.fcode = static_cast<const int32_t*>(h->at(h->lay.off_fcode));
  args.mat = h->lay.mat_bytes ? h->at(scaled ? h->lay.off_mat_dt : h->lay.off_mat) : nullptr;
  args.K = h->K;
  args.a = a;
  args.b = b;
  args.dt = dt;
  args.split_bf16 = h->prec == DG_BF16X3;
  args.wide_tiles = h->tile == 3;
  if (h->nscat) {
    args.src.rec = static_cast<const double*>(h->at(h->lay.off_src));
    args.src.phase = static_cast<const double*>(h->at(h->lay.off_phase));
    args.src.toff = toff;
  }
  HIP_TRY(dgk::launch_stage(h->N, h->f64(), stage, h->ops(), args, s));
  return DG_OK;
}

// One RK step's launches: five stages at t + c_i dt, then (scattered-field form) the device
// clock advances by dt. The caller advances the host mirror h->t.
int rk_step_launch(dg_handle* h, double dt, hipStream_t s) {
  for (int i = 0; i < 5; ++i) {
    int rc = stage_launch(h, true, h->u(h->cur), h->u(1 - h->cur), kRkA[i], kRkB[i], dt, s, kRkC[i] * dt);
    if (rc) return rc;
    h->cur ^= 1;
  }
  if (h->nscat) HIP_TRY(dgk::launch_advance_clock(static_cast<double*>(h->at(h->lay.off_src)), dt, s));
  return DG_OK;
}

int setup_impl(const dg_mesh* mesh, const dg_opts* opts, const std::vector<int32_t>* mesh_of,
               const std::vector<int32_t>* mesh_first, void* dev_workspace, size_t workspace_bytes,
               void* stream, dg_handle** out);

// The meshes of a batch as one mesh: vertex ids offset, elements and their face conditions
// and materials concatenated in mesh order.
struct Concat {
  std::vector<double> vxyz, eps, mu;
  std::vector<int32_t> etov, mesh_of, first;
  std::vector<int8_t> bc;
  dg_mesh m{};
};

int concat_meshes(const dg_mesh* meshes, int32_t count, Concat& c) {
  if (!meshes || count < 1) return fail(DG_E_ARG, "a batch needs at least one mesh");
  int64_t nv = 0, K = 0;
  bool any_bc = false, any_mat = false;
  for (int32_t i = 0; i < count; ++i) {
    const dg_mesh& m = meshes[i];
    if (!m.vxyz || !m.etov || m.K <= 0 || m.nverts < 4) return fail(DG_E_ARG, "empty or NULL mesh in the batch");
    nv += m.nverts;
    K += m.K;
    any_bc = any_bc || m.face_bc;
    any_mat = any_mat || m.eps || m.mu;
  }
  if (K >= (int64_t(1) << 26) || nv >= (int64_t(1) << 31)) return fail(DG_E_ARG, "batch too large");
  try {
    c.vxyz.reserve(size_t(nv) * 3);
    c.etov.reserve(size_t(K) * 4);
    c.first.push_back(0);
    int32_t vbase = 0;
    for (int32_t i = 0; i < count; ++i) {
      const dg_mesh& m = meshes[i];
      c.vxyz.insert(c.vxyz.end(), m.vxyz, m.vxyz + size_t(m.nverts) * 3);
      for (int64_t q = 0; q < int64_t(m.K) * 4; ++q) {
        const int32_t v = m.etov[q];
        if (v < 0 || v >= m.nverts) return fail(DG_E_MESH, "vertex id out of range");
        c.etov.push_back(v + vbase);
      }
      if (any_bc) {
        if (m.face_bc) c.bc.insert(c.bc.end(), m.face_bc, m.face_bc + size_t(m.K) * 4);
        else c.bc.insert(c.bc.end(), size_t(m.K) * 4, int8_t(0));
      }
      if (any_mat) {
        for (int k = 0; k < m.K; ++k) {
          c.eps.push_back(m.eps ? m.eps[k] : 1.0);
          c.mu.push_back(m.mu ? m.mu[k] : 1.0);
        }
      }
      c.mesh_of.insert(c.mesh_of.end(), size_t(m.K), i);
      c.first.push_back(c.first.back() + m.K);
      vbase += m.nverts;
    }
  } catch (const std::bad_alloc&) {
    return fail(DG_E_OOM, "host allocation failed");
  }
  c.m.nverts = int32_t(nv);
  c.m.vxyz = c.vxyz.data();
  c.m.K = int32_t(K);
  c.m.etov = c.etov.data();
  c.m.face_bc = any_bc ? c.bc.data() : nullptr;
  c.m.eps = any_mat ? c.eps.data() : nullptr;
  c.m.mu = any_mat ? c.mu.data() : nullptr;
  return DG_OK;
}

}  // namespace

extern "C" {

const char* dg_last_error(void) { return g_last_error.c_str(); }

int dg_setup_query(const dg_mesh* mesh, const dg_opts* opts, size_t* workspace_bytes) {
  int rc = check_inputs(mesh, opts);
  if (rc) return rc;
  if (!workspace_bytes) return fail(DG_E_ARG, "workspace_bytes must not be NULL");
  const int N = opts->order;
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  *workspace_bytes = make_layout(mesh->K, N, Np, Nfp, opts->precision, mesh->eps || mesh->mu, false,
                                 count_scatterers(mesh), opts->tile_id).total;
  return DG_OK;
}

int dg_setup(const dg_mesh* mesh, const dg_opts* opts, void* dev_workspace, size_t workspace_bytes,
             void* stream, dg_handle** out) {
  return setup_impl(mesh, opts, nullptr, nullptr, dev_workspace, workspace_bytes, stream, out);
}

}  // extern "C"

namespace {

// mesh_of (K or null): mesh id of each element of a concatenated batch; mesh_first: canonical
// element offsets of the meshes (count + 1 entries).
int setup_impl(const dg_mesh* mesh, const dg_opts* opts, const std::vector<int32_t>* mesh_of,
               const std::vector<int32_t>* mesh_first, void* dev_workspace, size_t workspace_bytes,
               void* stream, dg_handle** out) {
  if (out) *out = nullptr;
  if (!out) return fail(DG_E_ARG, "out must not be NULL");
  int rc = check_inputs(mesh, opts);
  if (rc) return rc;
  std::unique_ptr<dg_handle> h(new (std::nothrow) dg_handle);
  if (!h) return fail(DG_E_OOM, "host allocation failed");
  if (mesh_of) {
    h->batch = true;
    h->mesh_of = *mesh_of;
    h->mesh_first = *mesh_first;
  }
  try {
    h->ref = dgh::build_ref_ops(opts->order);
    h->mesh = dgh::build_mesh(h->ref, mesh->nverts, mesh->vxyz, mesh->K, mesh->etov, mesh->face_bc,
                              opts->reorder, mesh_of ? mesh_of->data() : nullptr);
  } catch (const std::bad_alloc&) {
    return fail(DG_E_OOM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(DG_E_MESH, ex.what());
  }
  if (mesh->eps || mesh->mu) {
    try {
      h->mat = dgh::material_records(h->mesh, mesh->eps, mesh->mu);
    } catch (const std::bad_alloc&) {
      return fail(DG_E_OOM, "host allocation failed");
    } catch (const std::exception& ex) {
      return fail(DG_E_ARG, ex.what());
    }
  }
  h->N = opts->order;
  h->Np = h->ref.Np;
  h->Nfp = h->ref.Nfp;
  h->K = mesh->K;
  h->prec = opts->precision;
  h->ts = h->f64() ? 8 : 4;
  h->S = dgk::row_stride(h->N, h->f64());
  h->device = opts->device;
  h->checks = opts->checks;
  h->nscat = int64_t(h->mesh.scat_face.size());
  if (h->nscat && h->batch) return fail(DG_E_UNSUPPORTED, "scatterer faces are not supported in a batch");
  h->lay = make_layout(h->K, h->N, h->Np, h->Nfp, h->prec, !h->mat.empty(), h->batch, h->nscat, opts->tile_id);
  h->tile = resolve_tile(h->N, h->prec, opts->tile_id);
  if (h->device >= 0) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = set_device(h.get());
    if (rc) return rc;
    // device address of the allocation-free call's scratch array, once per device
    HIP_TRY(dgk::noalloc_scratch_init(h->device));
    if (dev_workspace) {
      if (workspace_bytes < h->lay.total) return fail(DG_E_OOM, "workspace smaller than dg_setup_query");
      if (reinterpret_cast<uintptr_t>(dev_workspace) % 256 != 0)
        return fail(DG_E_ARG, "workspace must be 256-byte aligned");
      h->ws = static_cast<char*>(dev_workspace);
    } else {
      void* p = nullptr;
      hipError_t e = hipMalloc(&p, h->lay.total);
      if (e != hipSuccess) return fail(DG_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
      h->ws = static_cast<char*>(p);
      h->own_ws = true;
    }
    rc = upload(h.get(), s);
    if (rc) {
      if (h->own_ws) (void)hipFree(h->ws);
      return rc;
    }
    hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      if (h->own_ws) (void)hipFree(h->ws);
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
  }
  *out = h.release();
  return DG_OK;
}

}  // namespace

namespace {

// nsteps RK steps from the captured two-step graph of the current ping-pong parity (captured on
// first use or when dt changes), plus one plain step for an odd count; advances the host clock.
int solve_launch(dg_handle* h, double dt, int64_t nsteps, hipStream_t s) {
  if (nsteps >= 2) {
    // Two steps (ten stages) return the ping-pong state buffers to their starting roles, so
    // one captured graph per starting parity replays any even number of steps.
    const int p = h->cur;
    if (!h->gexec[p] || h->graph_dt[p] != dt) {
      h->drop_graph(p);
      const int saved = h->cur;
      HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      int r1 = rk_step_launch(h, dt, h->cap_stream);
      int r2 = r1 ? r1 : rk_step_launch(h, dt, h->cap_stream);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
      h->cur = saved;
      if (r2) {
        if (g) (void)hipGraphDestroy(g);
        return r2;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
      h->graph[p] = g;
      HIP_TRY(hipGraphInstantiate(&h->gexec[p], g, nullptr, nullptr, 0));
      h->graph_dt[p] = dt;
    }
    for (int64_t i = 0; i + 1 < nsteps; i += 2) {
      HIP_TRY(hipGraphLaunch(h->gexec[p], s));
      h->t += dt;
      h->t += dt;
    }
  }
  if (nsteps % 2) {
    int rc = rk_step_launch(h, dt, s);
    if (!rc) h->t += dt;
    return rc;
  }
  return DG_OK;
}

// Energy of the state, summed on the host in block order (synchronises s).
int energy_sync(const dg_handle* h, hipStream_t s, double* energy) {
  const int nb = (h->K + dgk::kEnergyBlockElems - 1) / dgk::kEnergyBlockElems;
  double* partial = static_cast<double*>(h->at(h->lay.off_partial));
  HIP_TRY(dgk::launch_energy(h->N, h->f64(), h->u(h->cur), h->ops().M, h->at(h->lay.off_geo),
                             h->lay.mat_bytes ? h->at(h->lay.off_mat) : nullptr, h->K, partial, s));
  std::vector<double> host(nb);
  HIP_TRY(hipMemcpyAsync(host.data(), partial, nb * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double e = 0.0;
  for (double v : host) e += v;
  *energy = e;
  return DG_OK;
}

}  // namespace

extern "C" {

int dg_free(dg_handle* h) {
  if (!h) return DG_OK;
  if (h->device >= 0) {
    (void)hipSetDevice(h->device);
    h->drop_graphs();
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    if (h->own_ws && h->ws) (void)hipFree(h->ws);
  }
  delete h;
  return DG_OK;
}

int dg_info(const dg_handle* h, dg_info_t* info) {
  if (!h || !info) return fail(DG_E_ARG, "NULL argument");
  info->order = h->N;
  info->Np = h->Np;
  info->Nfp = h->Nfp;
  info->K = h->K;
  info->precision = h->prec;
  info->device = h->device;
  info->state_words = int64_t(6) * h->K * h->Np;
  info->workspace_bytes = h->lay.total;
  return DG_OK;
}

int dg_nodes(const dg_handle* h, double* xyz) {
  if (!h || !xyz) return fail(DG_E_ARG, "NULL argument");
  std::memcpy(xyz, h->mesh.x.data(), h->mesh.x.size() * sizeof(double));
  return DG_OK;
}

int dg_get_maps(const dg_handle* h, int32_t* vmapM, int32_t* vmapP) {
  if (!h || !vmapM || !vmapP) return fail(DG_E_ARG, "NULL argument");
  dgh::canonical_maps(h->ref, h->mesh, vmapM, vmapP);
  return DG_OK;
}

int dg_get_operators(const dg_handle* h, double* Dr, double* Ds, double* Dt, double* LIFT, double* M,
                     double* rst) {
  if (!h) return fail(DG_E_ARG, "NULL handle");
  const auto& R = h->ref;
  if (Dr) std::copy(R.Dr.begin(), R.Dr.end(), Dr);
  if (Ds) std::copy(R.Ds.begin(), R.Ds.end(), Ds);
  if (Dt) std::copy(R.Dt.begin(), R.Dt.end(), Dt);
  if (LIFT) std::copy(R.LIFT.begin(), R.LIFT.end(), LIFT);
  if (M) std::copy(R.M.begin(), R.M.end(), M);
  if (rst)
    for (int n = 0; n < R.Np; ++n) rst[3 * n] = R.r[n], rst[3 * n + 1] = R.s[n], rst[3 * n + 2] = R.t[n];
  return DG_OK;
}

int dg_set_fields(dg_handle* h, const void* u, int on_device, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!u) return fail(DG_E_ARG, "NULL field array");
  rc = set_device(h);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const void* src = u;
  if (!on_device) {
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_tmp), u, h->lay.state, hipMemcpyHostToDevice, s));
    src = h->at(h->lay.off_tmp);
  }
  HIP_TRY(dgk::launch_to_internal(h->N, h->f64(), src, h->u(h->cur),
                                  static_cast<const int32_t*>(h->at(h->lay.off_pos_of)), h->K, s));
  HIP_TRY(dgk::launch_zero(h->at(h->lay.off_res), h->lay.istate, s));
  if (!on_device) HIP_TRY(hipStreamSynchronize(s));
  return DG_OK;
}

int dg_get_fields(const dg_handle* h, void* u, int on_device, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!u) return fail(DG_E_ARG, "NULL field array");
  rc = set_device(h);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* dst = on_device ? u : h->at(h->lay.off_tmp);
  HIP_TRY(dgk::launch_to_canonical(h->N, h->f64(), h->u(h->cur), dst,
                                   static_cast<const int32_t*>(h->at(h->lay.off_pos_of)), h->K, s));
  if (!on_device) {
    HIP_TRY(hipMemcpyAsync(u, dst, h->lay.state, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return DG_OK;
}

int dg_rhs(dg_handle* h, const void* u_dev, void* rhs_dev, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!u_dev || !rhs_dev || u_dev == rhs_dev) return fail(DG_E_ARG, "u and rhs must be distinct device arrays");
  rc = set_device(h);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  void* in = h->u(1 - h->cur);  // the spare state buffer is free between steps
  void* out = h->at(h->lay.off_tmp);
  HIP_TRY(dgk::launch_to_internal(h->N, h->f64(), u_dev, in, static_cast<const int32_t*>(h->at(h->lay.off_pos_of)),
                                  h->K, s));
  rc = stage_launch(h, false, in, out, 0, 0, 0, s);
  if (rc) return rc;
  HIP_TRY(dgk::launch_to_canonical(h->N, h->f64(), out, rhs_dev, static_cast<const int32_t*>(h->at(h->lay.off_pos_of)),
                                   h->K, s));
  return DG_OK;
}

int dg_rk_step(dg_handle* h, double dt, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!std::isfinite(dt)) return fail(DG_E_ARG, "dt must be finite");
  rc = set_device(h);
  if (rc) return rc;
  rc = rk_step_launch(h, dt, static_cast<hipStream_t>(stream));
  if (!rc) h->t += dt;
  return rc;
}

int dg_solve(dg_handle* h, double dt, int64_t nsteps, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!std::isfinite(dt) || nsteps < 0) return fail(DG_E_ARG, "bad dt or nsteps");
  rc = set_device(h);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (h->checks <= 0 || nsteps == 0) return solve_launch(h, dt, nsteps, s);
  // numeric monitor: chunks of `checks` steps, each followed by an energy check
  double e0 = 0.0;
  rc = energy_sync(h, s, &e0);
  if (rc) return rc;
  if (!std::isfinite(e0)) return fail(DG_E_NUMERIC, "non-finite energy before the first step");
  const double tol = h->f64() ? 1e-10 : 1e-4;
  for (int64_t done = 0; done < nsteps;) {
    const int64_t n = std::min<int64_t>(h->checks, nsteps - done);
    rc = solve_launch(h, dt, n, s);
    if (rc) return rc;
    done += n;
    double e1 = 0.0;
    rc = energy_sync(h, s, &e1);
    if (rc) return rc;
    if (!std::isfinite(e1))
      return fail(DG_E_NUMERIC, "non-finite energy after " + std::to_string(done) + " steps");
    if (h->nscat == 0 && e1 > e0 * (1.0 + tol))
      return fail(DG_E_NUMERIC, "energy grew from " + std::to_string(e0) + " to " + std::to_string(e1) + " in " +
                                    std::to_string(done) + " steps");
  }
  return DG_OK;
}

int dg_energy(const dg_handle* h, double* energy, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!energy) return fail(DG_E_ARG, "NULL energy");
  rc = set_device(h);
  if (rc) return rc;
  return energy_sync(h, static_cast<hipStream_t>(stream), energy);
}

int dg_energy_noalloc(const dg_handle* h, double* energy_dev, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!energy_dev) return fail(DG_E_ARG, "NULL energy_dev");
  const int64_t nb = (int64_t(h->K) + dgk::kEnergyBlockElems - 1) / dgk::kEnergyBlockElems;
  if (nb > dgk::kNoallocPartials)
    return fail(DG_E_ARG, "dg_energy_noalloc: K = " + std::to_string(h->K) + " exceeds the limit of " +
                              std::to_string(int64_t(dgk::kNoallocPartials) * dgk::kEnergyBlockElems) +
                              " elements (use dg_energy)");
  rc = set_device(h);
  if (rc) return rc;
  double* part = dgk::noalloc_scratch(h->device);
  if (!part) return fail(DG_E_STATE, "dg_energy_noalloc: scratch array not set up on this device");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(dgk::launch_energy(h->N, h->f64(), h->u(h->cur), h->ops().M, h->at(h->lay.off_geo),
                             h->lay.mat_bytes ? h->at(h->lay.off_mat) : nullptr, h->K, part, s));
  HIP_TRY(dgk::launch_sum(part, int(nb), energy_dev, s));
  return DG_OK;
}

int dg_set_incident(dg_handle* h, const double* k, const double* p, const double* profile, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!h->nscat) return fail(DG_E_ARG, "the mesh has no scatterer faces (face_bc = 3)");
  if (!k || !p || !profile) return fail(DG_E_ARG, "NULL argument");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(k[i]) || !std::isfinite(p[i])) return fail(DG_E_ARG, "k and p must be finite");
  for (int i = 0; i < 5; ++i)
    if (!std::isfinite(profile[i])) return fail(DG_E_ARG, "profile coefficients must be finite");
  const double kn = std::sqrt(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  if (!(kn > 0.0)) return fail(DG_E_ARG, "k must not be zero");
  const double kh[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
  const double pn = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  if (std::fabs(kh[0] * p[0] + kh[1] * p[1] + kh[2] * p[2]) > 1e-9 * std::max(pn, 1e-300))
    return fail(DG_E_ARG, "the polarisation p must be orthogonal to k");
  rc = set_device(h);
  if (rc) return rc;
  // phase k.x at the face nodes of each scatterer face, from the FP64 node coordinates
  const int Np = h->Np, Nfp = h->Nfp, K = h->K;
  std::vector<double> ph(size_t(h->nscat) * Nfp);
  for (int64_t i = 0; i < h->nscat; ++i) {
    const int32_t sf = h->mesh.scat_face[size_t(i)];
    const int ue = h->mesh.elem_of[sf / 4], f = sf % 4;
    for (int j = 0; j < Nfp; ++j) {
      const size_t n = size_t(ue) * Np + h->ref.Fmask[size_t(f) * Nfp + j];
      const size_t KN = size_t(K) * Np;
      ph[size_t(i) * Nfp + j] = kh[0] * h->mesh.x[n] + kh[1] * h->mesh.x[KN + n] + kh[2] * h->mesh.x[2 * KN + n];
    }
  }
  const double rec[dgk::kSrcRecWords] = {p[0], p[1], p[2], profile[0], profile[1], profile[2], profile[3],
                                         profile[4], h->t};
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_phase), ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_src), rec, sizeof(rec), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));   // host staging buffers die at return
  return DG_OK;
}

int dg_set_time(dg_handle* h, double t, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!std::isfinite(t)) return fail(DG_E_ARG, "t must be finite");
  rc = set_device(h);
  if (rc) return rc;
  if (h->nscat)
    HIP_TRY(dgk::launch_set_clock(static_cast<double*>(h->at(h->lay.off_src)), t, static_cast<hipStream_t>(stream)));
  h->t = t;
  return DG_OK;
}

int dg_get_time(const dg_handle* h, double* t) {
  if (!h || !t) return fail(DG_E_ARG, "NULL argument");
  *t = h->t;
  return DG_OK;
}

int dg_stable_dt(const dg_handle* h, double cfl, double* dt) {
  if (!h || !dt) return fail(DG_E_ARG, "NULL argument");
  double mn = 1e300;
  for (int k = 0; k < h->K; ++k)
    for (int f = 0; f < 4; ++f)
      mn = std::min(mn, 1.0 / h->mesh.geo[size_t(k) * dgh::kGeoStride + dgh::kGeoNormal + 4 * f + 3]);
  *dt = cfl * mn / (double(h->N) * h->N);
  return DG_OK;
}

int dg_setup_query_batch(const dg_mesh* meshes, int32_t count, const dg_opts* opts, size_t* workspace_bytes) {
  Concat c;
  int rc = concat_meshes(meshes, count, c);
  if (rc) return rc;
  rc = check_inputs(&c.m, opts);
  if (rc) return rc;
  if (!workspace_bytes) return fail(DG_E_ARG, "workspace_bytes must not be NULL");
  const int N = opts->order;
  const int Np = (N + 1) * (N + 2) * (N + 3) / 6, Nfp = (N + 1) * (N + 2) / 2;
  *workspace_bytes = make_layout(c.m.K, N, Np, Nfp, opts->precision, c.m.eps != nullptr, true, 0, opts->tile_id).total;
  return DG_OK;
}

int dg_setup_batch(const dg_mesh* meshes, int32_t count, const dg_opts* opts, void* dev_workspace,
                   size_t workspace_bytes, void* stream, dg_handle** out) {
  if (out) *out = nullptr;
  Concat c;
  int rc = concat_meshes(meshes, count, c);
  if (rc) return rc;
  return setup_impl(&c.m, opts, &c.mesh_of, &c.first, dev_workspace, workspace_bytes, stream, out);
}

int dg_batch_info(const dg_handle* h, int32_t* count, int32_t* first) {
  if (!h || !count) return fail(DG_E_ARG, "NULL argument");
  if (!h->batch) {
    *count = 1;
    if (first) first[0] = 0, first[1] = h->K;
    return DG_OK;
  }
  *count = int32_t(h->mesh_first.size()) - 1;
  if (first) std::copy(h->mesh_first.begin(), h->mesh_first.end(), first);
  return DG_OK;
}

int dg_batch_stable_dt(const dg_handle* h, double cfl, double* dt) {
  if (!h || !dt) return fail(DG_E_ARG, "NULL argument");
  const int count = h->batch ? int(h->mesh_first.size()) - 1 : 1;
  for (int i = 0; i < count; ++i) dt[i] = 1e300;
  for (int k = 0; k < h->K; ++k) {
    const int i = h->batch ? h->mesh_of[k] : 0;
    for (int f = 0; f < 4; ++f)
      dt[i] = std::min(dt[i], 1.0 / h->mesh.geo[size_t(k) * dgh::kGeoStride + dgh::kGeoNormal + 4 * f + 3]);
  }
  for (int i = 0; i < count; ++i) dt[i] *= cfl / (double(h->N) * h->N);
  return DG_OK;
}

int dg_set_batch_dt(dg_handle* h, const double* dt, void* stream) {
  int rc = need_device(h);
  if (rc) return rc;
  if (!h->batch) return fail(DG_E_ARG, "not a batch handle");
  if (!dt) return fail(DG_E_ARG, "NULL dt");
  const int count = int(h->mesh_first.size()) - 1;
  for (int i = 0; i < count; ++i)
    if (!(std::isfinite(dt[i]) && dt[i] > 0.0)) return fail(DG_E_ARG, "time steps must be finite and positive");
  rc = set_device(h);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // scale the inverse-map derivatives and Fscale (the right-hand side is linear in them) and
  // the material face weights; normals, J and the material constants stay
  const int K = h->K;
  std::vector<double> geo(h->geo_int), mat(h->mat);
  for (int i = 0; i < K; ++i) {
    const double sc = dt[h->mesh_of[h->mesh.elem_of[i]]];
    double* g = &geo[size_t(i) * dgh::kGeoStride];
    for (int q = 0; q < 9; ++q) g[q] *= sc;
    for (int f = 0; f < 4; ++f) g[dgh::kGeoNormal + 4 * f + 3] *= sc;
    if (!mat.empty())
      for (int q = dgh::kMatFace; q < dgh::kMatStride; ++q) mat[size_t(i) * dgh::kMatStride + q] *= sc;
  }
  std::vector<char> geo_b = to_prec(geo, h->f64());
  HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_geo_dt), geo_b.data(), geo_b.size(), hipMemcpyHostToDevice, s));
  std::vector<char> mat_b;
  if (h->lay.mat_dt_bytes) {
    mat_b = to_prec(mat, h->f64());
    HIP_TRY(hipMemcpyAsync(h->at(h->lay.off_mat_dt), mat_b.data(), mat_b.size(), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(hipStreamSynchronize(s));   // host staging buffers die at return
  return DG_OK;
}

}  // extern "C"

struct dg_group {
  std::vector<dg_handle*> m;
  int device = 0;
  hipStream_t cap = nullptr;               // the capture's origin stream
  std::vector<hipEvent_t> ev;              // fork event, then one join event per member
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> parity;                 // members' ping-pong parity at capture
  std::vector<double> dt;                  // members' steps at capture
  void drop() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  }
};

extern "C" {

int dg_group_create(dg_handle* const* members, int32_t count, dg_group** out) {
  if (out) *out = nullptr;
  if (!out || !members || count < 1) return fail(DG_E_ARG, "a group needs at least one member");
  std::unique_ptr<dg_group> g(new (std::nothrow) dg_group);
  if (!g) return fail(DG_E_OOM, "host allocation failed");
  for (int32_t i = 0; i < count; ++i) {
    dg_handle* h = members[i];
    int rc = need_device(h);
    if (rc) return rc;
    if (i && h->device != members[0]->device) return fail(DG_E_ARG, "group members must share a device");
    for (int32_t j = 0; j < i; ++j)
      if (members[j] == h) return fail(DG_E_ARG, "a handle appears twice in the group");
    g->m.push_back(h);
  }
  g->device = members[0]->device;
  int rc = set_device(members[0]);
  if (rc) return rc;
  g->ev.assign(size_t(count) + 1, nullptr);
  hipError_t e = hipStreamCreateWithFlags(&g->cap, hipStreamNonBlocking);
  for (auto& x : g->ev)
    if (e == hipSuccess) e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
  if (e != hipSuccess) {
    for (auto& x : g->ev)
      if (x) (void)hipEventDestroy(x);
    if (g->cap) (void)hipStreamDestroy(g->cap);
    return hip_fail(e, "dg_group_create");
  }
  *out = g.release();
  return DG_OK;
}

int dg_group_free(dg_group* g) {
  if (!g) return DG_OK;
  (void)hipSetDevice(g->device);
  g->drop();
  for (auto& x : g->ev)
    if (x) (void)hipEventDestroy(x);
  if (g->cap) (void)hipStreamDestroy(g->cap);
  delete g;
  return DG_OK;
}

int dg_group_solve(dg_group* g, const double* dt, int64_t nsteps, void* stream) {
  if (!g || !dt || nsteps < 0) return fail(DG_E_ARG, "bad group, dt or nsteps");
  const size_t n = g->m.size();
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(dt[i])) return fail(DG_E_ARG, "dt must be finite");
  HIP_TRY(hipSetDevice(g->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (nsteps >= 2) {
    bool same = g->gexec != nullptr;
    for (size_t i = 0; i < n && same; ++i) same = g->parity[i] == g->m[i]->cur && g->dt[i] == dt[i];
    if (!same) {
      g->drop();
      std::vector<int> saved(n);
      for (size_t i = 0; i < n; ++i) saved[i] = g->m[i]->cur;
      HIP_TRY(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
      int rc = 0;
      hipError_t e = hipEventRecord(g->ev[0], g->cap);
      for (size_t i = 0; i < n && !rc && e == hipSuccess; ++i) {
        dg_handle* h = g->m[i];
        e = hipStreamWaitEvent(h->cap_stream, g->ev[0], 0);
        if (e != hipSuccess) break;
        rc = rk_step_launch(h, dt[i], h->cap_stream);
        if (!rc) rc = rk_step_launch(h, dt[i], h->cap_stream);
        if (!rc) e = hipEventRecord(g->ev[i + 1], h->cap_stream);
        if (!rc && e == hipSuccess) e = hipStreamWaitEvent(g->cap, g->ev[i + 1], 0);
      }
      hipGraph_t graph = nullptr;
      hipError_t e2 = hipStreamEndCapture(g->cap, &graph);
      for (size_t i = 0; i < n; ++i) g->m[i]->cur = saved[i];
      if (rc || e != hipSuccess || e2 != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        if (rc) return rc;
        return hip_fail(e != hipSuccess ? e : e2, "group capture");
      }
      g->graph = graph;
      HIP_TRY(hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0));
      g->parity = saved;
      g->dt.assign(dt, dt + n);
    }
    for (int64_t k = 0; k + 1 < nsteps; k += 2) {
      HIP_TRY(hipGraphLaunch(g->gexec, s));
      for (size_t i = 0; i < n; ++i) {
        g->m[i]->t += dt[i];
        g->m[i]->t += dt[i];
      }
    }
  }
  if (nsteps % 2)
    for (size_t i = 0; i < n; ++i) {
      int rc = rk_step_launch(g->m[i], dt[i], s);
      if (rc) return rc;
      g->m[i]->t += dt[i];
    }
  return DG_OK;
}

}  // extern "C"

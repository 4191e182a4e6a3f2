"""Python binding of libdg (include/dg.h): nodal DG Maxwell on tetrahedra on one MI355X.

Argument marshalling only: every step of the operator runs in the library's HIP kernels.
PyTorch supplies device memory (the workspace and field buffers) and the HIP stream. The
library must have been built (`python -m paper_0901_1024_amd.build`); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdg.so")

DG_F64 = 0
DG_F32 = 1
DG_E_ARG = -1
DG_BF16X3 = 2
_PREC = {"f64": DG_F64, "f32": DG_F32, "bf16x3": DG_BF16X3}
_ERRS = {-1: "DG_E_ARG", -2: "DG_E_MESH", -3: "DG_E_UNSUPPORTED", -4: "DG_E_OOM", -5: "DG_E_HIP",
         -6: "DG_E_STATE", -7: "DG_E_NUMERIC"}

# every symbol declared in include/dg.h
EXPORTS = ["dg_setup_query", "dg_setup", "dg_free", "dg_last_error", "dg_info", "dg_nodes",
           "dg_get_maps", "dg_get_operators", "dg_set_fields", "dg_get_fields", "dg_rhs",
           "dg_rk_step", "dg_solve", "dg_energy", "dg_energy_noalloc", "dg_stable_dt", "dg_setup_query_batch",
           "dg_setup_batch", "dg_batch_info", "dg_batch_stable_dt", "dg_set_batch_dt", "dg_set_incident",
           "dg_set_time", "dg_get_time", "dg_group_create", "dg_group_free", "dg_group_solve"]


class DGError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRS.get(code, code)}: {msg}")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("nverts", ctypes.c_int32), ("vxyz", ctypes.POINTER(ctypes.c_double)),
                ("K", ctypes.c_int32), ("etov", ctypes.POINTER(ctypes.c_int32)),
                ("face_bc", ctypes.POINTER(ctypes.c_int8)), ("eps", ctypes.POINTER(ctypes.c_double)),
                ("mu", ctypes.POINTER(ctypes.c_double))]


class _Opts(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("precision", ctypes.c_int32), ("reorder", ctypes.c_int32),
                ("device", ctypes.c_int32), ("checks", ctypes.c_int32), ("tile_id", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class _Info(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("Np", ctypes.c_int32), ("Nfp", ctypes.c_int32),
                ("K", ctypes.c_int32), ("precision", ctypes.c_int32), ("device", ctypes.c_int32),
                ("state_words", ctypes.c_int64), ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """The loaded libdg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime (same SONAME as /opt/rocm's, requested under another
        # name). Loading torch first makes libdg bind to that one runtime instead of bringing a
        # second HIP/HSA runtime into the process, which would not see the device.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_0901_1024_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.dg_last_error.restype = ctypes.c_char_p
        L.dg_setup_query.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_size_t)]
        L.dg_setup.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Opts), vp, ctypes.c_size_t, vp,
                               ctypes.POINTER(vp)]
        L.dg_free.argtypes = [vp]
        L.dg_info.argtypes = [vp, ctypes.POINTER(_Info)]
        L.dg_nodes.argtypes = [vp, vp]
        L.dg_get_maps.argtypes = [vp, vp, vp]
        L.dg_get_operators.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.dg_set_fields.argtypes = [vp, vp, i32, vp]
        L.dg_get_fields.argtypes = [vp, vp, i32, vp]
        L.dg_rhs.argtypes = [vp, vp, vp, vp]
        L.dg_rk_step.argtypes = [vp, dbl, vp]
        L.dg_solve.argtypes = [vp, dbl, i64, vp]
        L.dg_energy.argtypes = [vp, ctypes.POINTER(dbl), vp]
        L.dg_energy_noalloc.argtypes = [vp, vp, vp]
        L.dg_stable_dt.argtypes = [vp, dbl, ctypes.POINTER(dbl)]
        L.dg_setup_query_batch.argtypes = [ctypes.POINTER(_Mesh), i32, ctypes.POINTER(_Opts),
                                           ctypes.POINTER(ctypes.c_size_t)]
        L.dg_setup_batch.argtypes = [ctypes.POINTER(_Mesh), i32, ctypes.POINTER(_Opts), vp, ctypes.c_size_t, vp,
                                     ctypes.POINTER(vp)]
        L.dg_batch_info.argtypes = [vp, ctypes.POINTER(i32), vp]
        L.dg_batch_stable_dt.argtypes = [vp, dbl, vp]
        L.dg_set_batch_dt.argtypes = [vp, vp, vp]
        L.dg_set_incident.argtypes = [vp, vp, vp, vp, vp]
        L.dg_set_time.argtypes = [vp, dbl, vp]
        L.dg_get_time.argtypes = [vp, ctypes.POINTER(dbl)]
        L.dg_group_create.argtypes = [vp, i32, ctypes.POINTER(vp)]
        L.dg_group_free.argtypes = [vp]
        L.dg_group_solve.argtypes = [vp, vp, i64, vp]
        for name in EXPORTS:
            if name != "dg_last_error":
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise DGError(rc, lib().dg_last_error().decode())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _mesh_struct(vxyz, etov, face_bc=None, eps=None, mu=None):
    vxyz = np.ascontiguousarray(vxyz, dtype=np.float64)
    etov = np.ascontiguousarray(etov, dtype=np.int32)
    m = _Mesh()
    m.nverts = vxyz.shape[0]
    m.vxyz = _ptr(vxyz, ctypes.c_double)
    m.K = etov.shape[0]
    m.etov = _ptr(etov, ctypes.c_int32)
    keep = [vxyz, etov]
    if face_bc is not None:
        fb = np.ascontiguousarray(face_bc, dtype=np.int8)
        if fb.shape != (m.K, 4):
            raise DGError(DG_E_ARG, "face_bc must have shape (K, 4)")
        m.face_bc = _ptr(fb, ctypes.c_int8)
        keep.append(fb)
    for name, arr in (("eps", eps), ("mu", mu)):
        if arr is not None:
            a = np.ascontiguousarray(arr, dtype=np.float64)
            if a.shape != (m.K,):
                raise DGError(DG_E_ARG, f"{name} must have shape (K,)")
            setattr(m, name, _ptr(a, ctypes.c_double))
            keep.append(a)
    return m, keep


def _opts_struct(order, precision, reorder, device, checks=0, tile_id=0):
    o = _Opts()
    o.order = order
    o.precision = _PREC[precision] if isinstance(precision, str) else int(precision)
    o.reorder = reorder
    o.device = device
    o.checks = checks
    o.tile_id = tile_id
    return o


def _tile_option(tile_id, order, precision, K):
    """tile_id: None or 0 = the library's default kernel, 1 = element-wise, 2 = contraction,
    3 = contraction with 16-element tiles (FP32 N = 3), "auto" = the autotuner's choice for this
    order, precision and mesh size (paper_0901_1024_amd.tune; the default when its table has no
    entry)."""
    if tile_id is None:
        return 0
    if tile_id == "auto":
        from . import tune
        return tune.choose(order, precision, K)
    return int(tile_id)


def setup_query(vxyz, etov, order, precision="f64", reorder=1, eps=None, mu=None, face_bc=None):
    m, _keep = _mesh_struct(vxyz, etov, face_bc=face_bc, eps=eps, mu=mu)
    o = _opts_struct(order, precision, reorder, 0)
    n = ctypes.c_size_t()
    _check(lib().dg_setup_query(ctypes.byref(m), ctypes.byref(o), ctypes.byref(n)))
    return n.value


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One mesh, one order (1..9), one precision ("f64", "f32", "bf16x3"): a handle of libdg.

    device >= 0: the workspace is a torch uint8 tensor on cuda:device (PyTorch owns the HBM);
    device = -1: host-only handle (builder outputs only).
    face_bc: (K, 4) int8, 0 automatic, 1 wall, 2 absorbing, 3 scatterer; eps, mu: (K,) per
    element; checks: numeric monitor interval of solve() in steps (0 = off); tile_id: stage
    kernel choice (see _tile_option).
    """

    def __init__(self, vxyz, etov, order, precision="f64", reorder=1, device=0, face_bc=None,
                 stream=None, eps=None, mu=None, checks=0, tile_id=None):
        L = lib()
        m, keep = _mesh_struct(vxyz, etov, face_bc, eps, mu)
        self._checks = checks
        self._tile = _tile_option(tile_id, order, precision, np.asarray(etov).shape[0])
        self._create(order, precision, reorder, device, stream,
                     lambda o, n: L.dg_setup_query(ctypes.byref(m), ctypes.byref(o), n),
                     lambda o, ws, n, s, h: L.dg_setup(ctypes.byref(m), ctypes.byref(o), ws, n, s, h))
        del keep

    def _create(self, order, precision, reorder, device, stream, query, setup):
        L = lib()
        self.order = order
        self.precision = precision
        self.device = device
        o = _opts_struct(order, precision, reorder, device, getattr(self, "_checks", 0), getattr(self, "_tile", 0))
        h = ctypes.c_void_p()
        self._ws = None
        if device >= 0:
            import torch
            n = ctypes.c_size_t()
            _check(query(o, ctypes.byref(n)))
            with torch.cuda.device(device):
                self._ws = torch.empty(n.value + 256, dtype=torch.uint8, device=f"cuda:{device}")
                base = self._ws.data_ptr()
                aligned = (base + 255) & ~255
                _check(setup(o, ctypes.c_void_p(aligned), ctypes.c_size_t(n.value), _stream_ptr(stream),
                             ctypes.byref(h)))
        else:
            _check(setup(o, None, 0, None, ctypes.byref(h)))
        self._h = h
        info = _Info()
        _check(L.dg_info(h, ctypes.byref(info)))
        self.Np, self.Nfp, self.K = info.Np, info.Nfp, info.K
        self.workspace_bytes = info.workspace_bytes
        self.dtype = np.float64 if o.precision == DG_F64 else np.float32

    # -- lifecycle -------------------------------------------------------------------------
    def free(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().dg_free(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    # -- host outputs ----------------------------------------------------------------------
    def nodes(self):
        out = np.empty((3, self.K, self.Np), dtype=np.float64)
        _check(lib().dg_nodes(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def get_maps(self):
        vM = np.empty((self.K, 4, self.Nfp), dtype=np.int32)
        vP = np.empty_like(vM)
        _check(lib().dg_get_maps(self._h, vM.ctypes.data_as(ctypes.c_void_p), vP.ctypes.data_as(ctypes.c_void_p)))
        return vM, vP

    def get_operators(self):
        Np, Nfp = self.Np, self.Nfp
        Dr, Ds, Dt, M = (np.empty((Np, Np)) for _ in range(4))
        LIFT = np.empty((Np, 4 * Nfp))
        rst = np.empty((Np, 3))
        vp = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().dg_get_operators(self._h, vp(Dr), vp(Ds), vp(Dt), vp(LIFT), vp(M), vp(rst)))
        return {"Dr": Dr, "Ds": Ds, "Dt": Dt, "LIFT": LIFT, "M": M, "rst": rst}

    def stable_dt(self, cfl=0.5):
        d = ctypes.c_double()
        _check(lib().dg_stable_dt(self._h, cfl, ctypes.byref(d)))
        return d.value

    # -- device state ----------------------------------------------------------------------
    def set_fields(self, u, stream=None):
        """u: canonical (6, K, Np) array, numpy (host) or torch CUDA tensor of the working dtype."""
        if isinstance(u, np.ndarray):
            a = np.ascontiguousarray(u, dtype=self.dtype)
            assert a.size == 6 * self.K * self.Np
            _check(lib().dg_set_fields(self._h, a.ctypes.data_as(ctypes.c_void_p), 0, _stream_ptr(stream)))
        else:
            self._check_tensor(u)
            _check(lib().dg_set_fields(self._h, ctypes.c_void_p(u.data_ptr()), 1, _stream_ptr(stream)))

    def get_fields(self, out=None, stream=None):
        """Canonical (6, K, Np) fields: into `out` (torch CUDA tensor) or a new numpy array."""
        if out is None:
            a = np.empty((6, self.K, self.Np), dtype=self.dtype)
            _check(lib().dg_get_fields(self._h, a.ctypes.data_as(ctypes.c_void_p), 0, _stream_ptr(stream)))
            return a
        self._check_tensor(out)
        _check(lib().dg_get_fields(self._h, ctypes.c_void_p(out.data_ptr()), 1, _stream_ptr(stream)))
        return out

    def rhs(self, u, out, stream=None):
        """Right-hand side of canonical device tensor u into canonical device tensor out."""
        self._check_tensor(u)
        self._check_tensor(out)
        _check(lib().dg_rhs(self._h, ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                            _stream_ptr(stream)))
        return out

    def rk_step(self, dt, stream=None):
        _check(lib().dg_rk_step(self._h, float(dt), _stream_ptr(stream)))

    def solve(self, dt, nsteps, stream=None):
        _check(lib().dg_solve(self._h, float(dt), int(nsteps), _stream_ptr(stream)))

    def energy(self, stream=None):
        e = ctypes.c_double()
        _check(lib().dg_energy(self._h, ctypes.byref(e), _stream_ptr(stream)))
        return e.value

    def set_incident(self, k, p, profile, stream=None):
        """Incident plane wave of the scattered-field form (dg_set_incident): direction k,
        polarisation p, profile f(s) = c0 + c1 s + c2 sin(c3 s + c4)."""
        k = np.ascontiguousarray(k, dtype=np.float64)
        p = np.ascontiguousarray(p, dtype=np.float64)
        c = np.ascontiguousarray(profile, dtype=np.float64)
        if k.shape != (3,) or p.shape != (3,) or c.shape != (5,):
            raise DGError(-1, "k, p need 3 values and the profile 5")
        _check(lib().dg_set_incident(self._h, k.ctypes.data_as(ctypes.c_void_p), p.ctypes.data_as(ctypes.c_void_p),
                                     c.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))

    def set_time(self, t, stream=None):
        _check(lib().dg_set_time(self._h, float(t), _stream_ptr(stream)))

    @property
    def time(self):
        t = ctypes.c_double()
        _check(lib().dg_get_time(self._h, ctypes.byref(t)))
        return t.value

    def energy_noalloc(self, out, stream=None):
        """dg_energy_noalloc: the energy into out[0] (a float64 CUDA tensor) on the stream,
        without allocating or synchronising."""
        import torch
        if not (out.is_cuda and out.dtype == torch.float64 and out.numel() >= 1 and out.is_contiguous()):
            raise DGError(-1, "expected a contiguous float64 CUDA tensor with at least one element")
        _check(lib().dg_energy_noalloc(self._h, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def _check_tensor(self, t):
        import torch
        want = torch.float64 if self.dtype == np.float64 else torch.float32
        if not (t.is_cuda and t.dtype == want and t.is_contiguous() and t.numel() == 6 * self.K * self.Np):
            raise DGError(-1, "expected a contiguous CUDA tensor of 6*K*Np values of the working dtype")


class BatchSolver(Solver):
    """Many meshes of one order and precision in one handle (the batched form).

    meshes: list of dicts with keys vxyz, etov and optionally face_bc, eps, mu. Canonical field
    arrays are the meshes' arrays concatenated along the element axis; mesh i owns elements
    first[i]:first[i+1]. Each mesh advances with its own step (set_dts); solve(1.0, n) then
    takes n steps of every mesh.
    """

    def __init__(self, meshes, order, precision="f64", reorder=1, device=0, stream=None, tile_id=None):
        L = lib()
        self._tile = _tile_option(tile_id, order, precision, sum(np.asarray(md["etov"]).shape[0] for md in meshes))
        arr = (_Mesh * len(meshes))()
        keep = []
        for i, md in enumerate(meshes):
            m, k = _mesh_struct(md["vxyz"], md["etov"], md.get("face_bc"), md.get("eps"), md.get("mu"))
            arr[i] = m
            keep.append(k)
        cnt = len(meshes)
        self._create(order, precision, reorder, device, stream,
                     lambda o, n: L.dg_setup_query_batch(arr, cnt, ctypes.byref(o), n),
                     lambda o, ws, n, s, h: L.dg_setup_batch(arr, cnt, ctypes.byref(o), ws, n, s, h))
        del keep
        c = ctypes.c_int32()
        _check(L.dg_batch_info(self._h, ctypes.byref(c), None))
        self.first = np.empty(c.value + 1, dtype=np.int32)
        _check(L.dg_batch_info(self._h, ctypes.byref(c), self.first.ctypes.data_as(ctypes.c_void_p)))
        self.count = c.value

    def stable_dts(self, cfl=0.5):
        out = np.empty(self.count)
        _check(lib().dg_batch_stable_dt(self._h, float(cfl), out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def set_dts(self, dts, stream=None):
        d = np.ascontiguousarray(dts, dtype=np.float64)
        if d.shape != (self.count,):
            raise DGError(DG_E_ARG, "one time step per mesh")
        _check(lib().dg_set_batch_dt(self._h, d.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))

    def mesh_slice(self, i):
        return slice(int(self.first[i]), int(self.first[i + 1]))


class Group:
    """Handles of any orders and precisions advanced together from one captured graph
    (dg_group_*): solve(dts, n) takes n steps of every member, member i with step dts[i]."""

    def __init__(self, solvers):
        L = lib()
        self.members = list(solvers)
        arr = (ctypes.c_void_p * len(self.members))(*[s._h.value for s in self.members])
        g = ctypes.c_void_p()
        _check(L.dg_group_create(arr, len(self.members), ctypes.byref(g)))
        self._g = g

    def solve(self, dts, nsteps, stream=None):
        d = np.ascontiguousarray(dts, dtype=np.float64)
        if d.shape != (len(self.members),):
            raise DGError(DG_E_ARG, "one time step per member")
        _check(lib().dg_group_solve(self._g, d.ctypes.data_as(ctypes.c_void_p), int(nsteps), _stream_ptr(stream)))

    def free(self):
        if getattr(self, "_g", None) is not None and self._g.value:
            lib().dg_group_free(self._g)
        self._g = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class MixedBatch:
    """The batched form over meshes of mixed orders: one batch handle per order (meshes of one
    order share its launches), all of them advanced by one group graph. Every mesh takes its
    own stable step (set_dts); fields are per-mesh canonical arrays."""

    def __init__(self, meshes, orders, precision="f32", reorder=1, device=0, stream=None, tile_id=None):
        self.orders = sorted(set(int(n) for n in orders))
        self.where = []                     # mesh -> (order index, position in that batch)
        groups = {n: [] for n in self.orders}
        for i, (md, n) in enumerate(zip(meshes, orders)):
            self.where.append((self.orders.index(int(n)), len(groups[int(n)])))
            groups[int(n)].append(md)
        self.batches = [BatchSolver(groups[n], n, precision, reorder, device, stream, tile_id) for n in self.orders]
        self.group = Group(self.batches)
        self.K = sum(b.K for b in self.batches)

    def stable_dts(self, cfl=0.5):
        per = [b.stable_dts(cfl) for b in self.batches]
        return np.array([per[o][j] for o, j in self.where])

    def set_dts(self, dts, stream=None):
        for o, b in enumerate(self.batches):
            d = np.empty(b.count)
            for i, (oo, j) in enumerate(self.where):
                if oo == o:
                    d[j] = dts[i]
            b.set_dts(d, stream)

    def set_fields(self, us, stream=None):
        for o, b in enumerate(self.batches):
            parts = [None] * b.count
            for i, (oo, j) in enumerate(self.where):
                if oo == o:
                    parts[j] = np.asarray(us[i], dtype=b.dtype)
            b.set_fields(np.concatenate(parts, axis=1), stream)

    def get_fields(self, stream=None):
        outs = [b.get_fields(stream=stream) for b in self.batches]
        return [outs[o][:, self.batches[o].mesh_slice(j)] for o, j in self.where]

    def solve(self, nsteps, stream=None):
        self.group.solve(np.ones(len(self.batches)), nsteps, stream)

    def free(self):
        self.group.free()
        for b in self.batches:
            b.free()

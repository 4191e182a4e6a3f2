"""Parity at full mesh sizes and on meshes that reach every face orientation.

The persistent FP32 contraction kernels give each workgroup several tiles only when the mesh
has more tiles than the resident grid; these meshes are that large, their last tile is
ragged, and their elements list their vertices in random order (all 48 face / neighbour-face
/ rotation combinations occur), so the steady-state loop (next-tile prefetch, exterior traces
gathered a tile ahead, face records double-buffered) runs against the oracle in vacuum and in
a medium with absorbing faces. The oracle evaluates the right-hand side at sampled elements
and one RK step at a few elements (their five-stage dependency cone).

Bounds: relative L2 over the sampled values (1e-5 in FP32, 1e-12 in FP64) and pointwise
max |a - b| / max |b| (1e-4 in FP32, 1e-11 in FP64).
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, face_combos, gpu_rhs, max_rel, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
_CACHE = {}


def big_problem(N, n):
    """Jittered, permuted, vertex-shuffled n^3 Kuhn cube at order N, with its smooth fields,
    random eps / mu and absorbing faces on z = 1 (cached per (N, n))."""
    key = (N, n)
    if key not in _CACHE:
        v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=True)
        m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
        u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32")
        eps, mu = dginputs.random_materials(m.K, seed=23)
        fb = dginputs.faces_on_plane(v, e, 2, 1.0) * 2
        absorb = dginputs.faces_on_plane(v, m.etov, 2, 1.0).astype(bool)
        _CACHE.clear()
        _CACHE[key] = (v, e, m, u, eps, mu, fb, absorb)
    return _CACHE[key]


def check_sampled(s, m, u, kw, prec, nsample, nstep, seed):
    g = np.random.default_rng(seed)
    boundary = np.nonzero(m.boundary.any(1))[0]
    sample = np.unique(np.concatenate([g.choice(m.K, nsample, replace=False),
                                       g.choice(boundary, 16, replace=False), [0, m.K - 1]]))
    r = gpu_rhs(s, u)
    ro = W.rhs_at(m, u, sample, **kw)
    err, mx = rel_l2(r[:, sample], ro), max_rel(r[:, sample], ro)
    say(f"  sampled rhs ({sample.size} elements) rel {err:.2e} max {mx:.2e}")
    assert err <= TOL[prec] and mx <= MAX_TOL[prec]
    dt = W.stable_dt(m)
    s.set_fields(u)
    s.rk_step(dt)
    ug = s.get_fields()
    step_sample = sample[:nstep]
    uo = W.lsrk4_step_at(m, u, dt, step_sample, **kw)
    err1, mx1 = rel_l2(ug[:, step_sample], uo), max_rel(ug[:, step_sample], uo)
    say(f"  sampled 1-step rel {err1:.2e} max {mx1:.2e}")
    assert err1 <= TOL[prec] and mx1 <= MAX_TOL[prec]


# (order, cube size n): K = 6 n^3 leaves a ragged last tile (16-element tiles at N = 4:
# 355,914 = 16 * 22,244 + 10; 8-element tiles at N = 3, 5, 6, 7: 355,914 = 8 * 44,489 + 2,
# 178,746 = 8 * 22,343 + 2 and 93,750 = 8 * 11,718 + 6), and every workgroup of the
# persistent grid takes many tiles (at N = 7 the operator strip is streamed per tile)
FULL = [(3, 39), (4, 39), (5, 31), (6, 31), (7, 25)]


@pytest.mark.parametrize("medium", [False, True])   # innermost: both variants share a mesh
@pytest.mark.parametrize("N,n", FULL)
def test_fp32_full_size_steady_state_loop(N, n, medium):
    v, e, m, u, eps, mu, fb, absorb = big_problem(N, n)
    if N == 4 and not medium:
        pytest.skip("vacuum N = 4 at full size is test_gpu_parity.test_fp32_full_size_n4_sampled")
    say(f"case: N={N} K={m.K} f32 full size, shuffled vertices, {'medium+absorbing' if medium else 'vacuum'}")
    kw = dict(eps=eps, mu=mu, absorb=absorb) if medium else {}
    s = P.Solver(v, e, N, "f32", reorder=1, **(dict(eps=eps, mu=mu, face_bc=fb) if medium else {}))
    check_sampled(s, m, u, kw, "f32", 700, 10, seed=100 + N)
    s.free()


@pytest.mark.parametrize("medium", [False, True])
@pytest.mark.parametrize("N,n", [(3, 39), (4, 31), (5, 31), (6, 31), (7, 25)])
def test_fp64_contraction_kernel_full_size(N, n, medium):
    """FP64 on its contraction kernels at full size, 8-element tiles with a ragged last one:
    N = 3 on 355,914 = 8 * 44,489 + 2 elements, N = 4 (padded LDS rows), 5 and 6 on 178,746 =
    8 * 22,343 + 2, N = 7 on 93,750 = 8 * 11,718 + 6 (every workgroup takes many tiles);
    vacuum and medium with absorbing faces."""
    v, e, m, u, eps, mu, fb, absorb = big_problem(N, n)
    say(f"case: N={N} K={m.K} f64 full size, shuffled vertices, {'medium+absorbing' if medium else 'vacuum'}")
    kw = dict(eps=eps, mu=mu, absorb=absorb) if medium else {}
    s = P.Solver(v, e, N, "f64", reorder=1, **(dict(eps=eps, mu=mu, face_bc=fb) if medium else {}))
    check_sampled(s, m, u, kw, "f64", 700, 10, seed=140 + N)
    s.free()


@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_all_face_orientations(N, prec):
    """Every (face, neighbour face, rotation) combination a conforming mesh allows, on every
    kernel: FP64 at all orders (the contraction kernel at N = 3); FP32 on the contraction
    kernels (N = 3..7) and the element-wise kernel (N = 1, 2). Whole-mesh right-hand side and
    one RK step."""
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True, shuffle=True)
    assert len(face_combos(v, e)) == 48
    m = Mm.Mesh(v, e, R.ref_element(N))
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), prec)
    say(f"case: N={N} K={m.K} {prec} shuffled vertices (48 orientation combinations)")
    s = P.Solver(v, e, N, prec)
    r, ro = gpu_rhs(s, u), W.rhs(m, u)
    assert rel_l2(r, ro) <= TOL[prec] and max_rel(r, ro) <= MAX_TOL[prec]
    dt = W.stable_dt(m)
    s.set_fields(u)
    s.rk_step(dt)
    uo, _ = W.lsrk4_step(m, u, dt)
    ug = s.get_fields()
    assert rel_l2(ug, uo) <= TOL[prec] and max_rel(ug, uo) <= MAX_TOL[prec]


@pytest.mark.parametrize("N,sizes", [(4, (12, 14, 9)), (6, (8, 7, 9))])
def test_batch_larger_than_the_resident_grid(N, sizes):
    """A batch handle of three shuffled meshes (one in a medium with absorbing faces) whose
    tiles outnumber the persistent grid, each mesh against the oracle (sampled right-hand
    side, and a sampled RK step at the mesh's own time step)."""
    meshes, oms = [], []
    for i, n in enumerate(sizes):
        v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=True, seed_jitter=40 + i,
                                  seed_perm=50 + i)
        md = {"vxyz": v, "etov": e}
        m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
        kw = {}
        if i == 1:
            md["eps"], md["mu"] = dginputs.random_materials(e.shape[0], seed=33)
            md["face_bc"] = dginputs.faces_on_plane(v, e, 2, 1.0) * 2
            kw = dict(eps=md["eps"], mu=md["mu"], absorb=dginputs.faces_on_plane(v, m.etov, 2, 1.0).astype(bool))
        meshes.append(md)
        oms.append((m, kw))
    b = P.BatchSolver(meshes, N, "f32")
    say(f"case: batch N={N} K={b.K} f32 (meshes {[md['etov'].shape[0] for md in meshes]})")
    us = [rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32") for m, _ in oms]
    ub = np.concatenate(us, axis=1)
    rb = gpu_rhs(b, ub)
    g = np.random.default_rng(60 + N)
    samples = []
    for i, (m, kw) in enumerate(oms):
        smp = np.unique(np.concatenate([g.choice(m.K, 200, replace=False), [0, m.K - 1]]))
        samples.append(smp)
        ro = W.rhs_at(m, us[i], smp, **kw)
        got = rb[:, b.mesh_slice(i)][:, smp]
        assert rel_l2(got, ro) <= TOL["f32"] and max_rel(got, ro) <= MAX_TOL["f32"], i
    dts = b.stable_dts(0.5)
    b.set_dts(dts)
    b.set_fields(ub)
    b.rk_step(1.0)
    got = b.get_fields()
    for i, (m, kw) in enumerate(oms):
        smp = samples[i][:6]
        uo = W.lsrk4_step_at(m, us[i], dts[i], smp, **kw)
        g1 = got[:, b.mesh_slice(i)][:, smp]
        err = rel_l2(g1, uo)
        say(f"  mesh {i}: K={m.K} dt={dts[i]:.3e} sampled 1-step rel {err:.2e}")
        assert err <= TOL["f32"] and max_rel(g1, uo) <= MAX_TOL["f32"]

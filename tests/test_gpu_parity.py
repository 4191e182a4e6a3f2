"""Parity of the HIP path (through the C ABI) with the FP64 oracle on seeded inputs.

Tolerances: relative discrete L2 over all fields and nodes, 1e-12 in FP64 and 1e-5 in FP32
(the FP32 oracle input is the FP32-rounded field cast back to FP64); face maps bit-exact.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, gpu_rhs, max_rel, per_field_rel, problem, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def test_cavity_n3_fp64_rhs_and_twenty_steps():
    """Unit cube 8^3 x 6 = 3072 tets, N = 3, FP64, (1,1,0) TM mode, dt at CFL 0.5, 20 steps."""
    say("case: cavity N=3 K=3072 f64")
    v, e, m, u0 = problem(3, 8, fields="cavity")
    s = P.Solver(v, e, 3, "f64", reorder=1)
    vM, vP = s.get_maps()
    assert np.array_equal(vM, m.vmapM) and np.array_equal(vP, m.vmapP)
    r = gpu_rhs(s, u0)
    ro = W.rhs(m, u0)
    assert rel_l2(r, ro) <= TOL["f64"]
    dt = W.stable_dt(m)
    assert abs(dt - s.stable_dt(0.5)) <= 1e-15 * dt
    s.set_fields(u0)
    e0 = s.energy()
    assert abs(e0 - W.energy(m, u0)) <= 1e-12 * e0
    s.solve(dt, 20)
    ug = s.get_fields()
    uo, res = u0, None
    for _ in range(20):
        uo, res = W.lsrk4_step(m, uo, dt, res)
    err = rel_l2(ug, uo)
    say("  rhs rel", rel_l2(r, ro), "20-step rel", err, "per field", per_field_rel(ug, uo))
    assert err <= TOL["f64"]
    e20 = s.energy()
    assert e20 <= e0 * (1 + 1e-14)
    assert abs(e20 - W.energy(m, uo)) <= 1e-12 * e0


@pytest.mark.parametrize("N", range(1, 10))
def test_all_orders_fp64_jittered_permuted(N):
    """162 tets (ragged last tile for every order), jittered and permuted, smooth fields."""
    say(f"case: N={N} K=162 f64 jitter+permute")
    v, e, m, u0 = problem(N, 3, jitter=0.15, permute=True)
    s = P.Solver(v, e, N, "f64", reorder=1)
    r, ro = gpu_rhs(s, u0), W.rhs(m, u0)
    assert rel_l2(r, ro) <= TOL["f64"] and max_rel(r, ro) <= MAX_TOL["f64"]
    dt = W.stable_dt(m)
    s.set_fields(u0)
    s.solve(dt, 3)
    uo, res = u0, None
    for _ in range(3):
        uo, res = W.lsrk4_step(m, uo, dt, res)
    ug = s.get_fields()
    assert rel_l2(ug, uo) <= TOL["f64"] and max_rel(ug, uo) <= MAX_TOL["f64"]


@pytest.mark.parametrize("N,n", [(2, 3), (3, 3), (4, 3), (4, 4), (5, 3), (5, 4), (6, 3), (6, 4), (7, 2),
                                 (8, 2), (9, 2)])
def test_fp32_orders_small_mesh(N, n):
    """K = 162 leaves a ragged last tile of every tile size; K = 384 fills them. N = 4 runs on
    the 16-element MFMA kernel, N = 3, 5, 6, 7 on 8-element ones, N = 2, 8, 9 on the VALU one."""
    say(f"case: N={N} K={6 * n ** 3} f32 jitter+permute")
    v, e, m, u0 = problem(N, n, jitter=0.15, permute=True)
    s = P.Solver(v, e, N, "f32", reorder=1)
    u32 = rounded(u0, "f32")
    r, ro = gpu_rhs(s, u32), W.rhs(m, u32)
    err = rel_l2(r, ro)
    say("  rhs rel", err, "max", max_rel(r, ro))
    assert err <= TOL["f32"] and max_rel(r, ro) <= MAX_TOL["f32"]
    dt = W.stable_dt(m)
    s.set_fields(u32)
    s.rk_step(dt)
    uo, _ = W.lsrk4_step(m, u32, dt)
    ug = s.get_fields()
    assert rel_l2(ug, uo) <= TOL["f32"] and max_rel(ug, uo) <= MAX_TOL["f32"]


def test_fp32_full_size_n4_sampled():
    """6 * 40^3 = 384,000 jittered, permuted tets, N = 4, FP32: the benchmark's workload and
    launch configuration. The oracle evaluates the right-hand side and one RK step at sampled
    elements only (dependency cone of the five stages)."""
    say("case: N=4 K=384000 f32 full size, sampled")
    v, e, m, u0 = problem(4, 40, jitter=0.15, permute=True, compute_maps=False)
    s = P.Solver(v, e, 4, "f32", reorder=1)
    u32 = rounded(u0, "f32")
    g = np.random.default_rng(11)
    sample = np.unique(np.concatenate([g.choice(m.K, 1500, replace=False), [0, m.K - 1]]))
    r = gpu_rhs(s, u32)
    ro = W.rhs_at(m, u32, sample)
    err = rel_l2(r[:, sample], ro)
    say("  sampled rhs rel", err, "max", max_rel(r[:, sample], ro), "per field", per_field_rel(r[:, sample], ro))
    assert err <= TOL["f32"] and max_rel(r[:, sample], ro) <= MAX_TOL["f32"]
    dt = W.stable_dt(m)
    s.set_fields(u32)
    e0 = s.energy()
    s.rk_step(dt)
    ug = s.get_fields()
    step_sample = sample[:24]
    uo = W.lsrk4_step_at(m, u32, dt, step_sample)
    err1 = rel_l2(ug[:, step_sample], uo)
    say("  sampled 1-step rel", err1)
    assert err1 <= TOL["f32"]
    assert s.energy() <= e0 * (1 + 1e-6)


def test_fp32_full_size_n5_sampled():
    """6 * 32^3 = 196,608 jittered, permuted tets, N = 5, FP32 (the 8-element MFMA kernel at the
    size of the precision sweep); sampled right-hand side and one RK step against the oracle."""
    say("case: N=5 K=196608 f32 full size, sampled")
    v, e, m, u0 = problem(5, 32, jitter=0.15, permute=True, compute_maps=False)
    s = P.Solver(v, e, 5, "f32", reorder=1)
    u32 = rounded(u0, "f32")
    g = np.random.default_rng(12)
    sample = np.unique(np.concatenate([g.choice(m.K, 800, replace=False), [0, m.K - 1]]))
    r = gpu_rhs(s, u32)
    err = rel_l2(r[:, sample], W.rhs_at(m, u32, sample))
    say("  sampled rhs rel", err)
    assert err <= TOL["f32"]
    dt = W.stable_dt(m)
    s.set_fields(u32)
    s.rk_step(dt)
    step_sample = sample[:12]
    err1 = rel_l2(s.get_fields()[:, step_sample], W.lsrk4_step_at(m, u32, dt, step_sample))
    say("  sampled 1-step rel", err1)
    assert err1 <= TOL["f32"]


def test_reorder_and_repeat_are_bitwise_identical():
    v, e, m, u0 = problem(4, 3, jitter=0.15, permute=True)
    a = P.Solver(v, e, 4, "f64", reorder=1)
    b = P.Solver(v, e, 4, "f64", reorder=0)
    ra, ra2, rb = gpu_rhs(a, u0), gpu_rhs(a, u0), gpu_rhs(b, u0)
    assert np.array_equal(ra, ra2)
    assert np.array_equal(ra, rb)
    dt = W.stable_dt(m)
    for s in (a, b):
        s.set_fields(u0)
        s.solve(dt, 4)
    assert np.array_equal(a.get_fields(), b.get_fields())


def test_solve_equals_repeated_steps_and_field_round_trip():
    import torch
    v, e, m, u0 = problem(3, 2, jitter=0.1, permute=True)
    s = P.Solver(v, e, 3, "f64")
    s.set_fields(u0)
    assert np.array_equal(s.get_fields(), u0)
    t = torch.from_numpy(u0).cuda()
    s.set_fields(t)
    back = torch.empty_like(t)
    s.get_fields(back)
    torch.cuda.synchronize()
    assert torch.equal(back, t)
    dt = W.stable_dt(m)
    s.solve(dt, 5)          # two graph replays and one plain step
    a = s.get_fields()
    s.set_fields(u0)
    for _ in range(5):
        s.rk_step(dt)
    assert np.array_equal(a, s.get_fields())
    s.set_fields(u0)
    s.solve(dt, 2)
    s.solve(dt, 3)
    assert np.array_equal(a, s.get_fields())


@pytest.mark.parametrize("N", [1, 3, 4, 5, 6, 7, 9])
def test_degenerate_meshes_single_and_two_tets(N):
    one_v = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    two_v = np.vstack([one_v, [[0.9, 0.8, 0.95]]])
    for v, e in ((one_v, np.array([[0, 1, 2, 3]])), (two_v, np.array([[0, 1, 2, 3], [1, 2, 3, 4]]))):
        m = Mm.Mesh(v, e, R.ref_element(N))
        x, y, z = m.x
        u0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x, y, z)
        s = P.Solver(v, e, N, "f64")
        assert rel_l2(gpu_rhs(s, u0), W.rhs(m, u0)) <= TOL["f64"]


@pytest.mark.parametrize("N", [3, 4, 5, 6])
def test_fp32_field_round_trip_and_energy(N):
    """The FP32 internal layout (rows padded to a multiple of 4 nodes at N = 4, pad words kept
    zero): fields come back bitwise through the host and the device paths, and the energy
    equals the oracle's for the same FP32 values, in vacuum and in a medium."""
    import torch
    v, e, m, u0 = problem(N, 3, jitter=0.15, permute=True)
    u32 = rounded(u0, "f32")
    eps, mu = dginputs.random_materials(e.shape[0])
    for kw in ({}, dict(eps=eps, mu=mu)):
        say(f"case: N={N} K={m.K} f32 {'medium' if kw else 'vacuum'} round trip + energy")
        s = P.Solver(v, e, N, "f32", reorder=1, **kw)
        s.set_fields(u32)
        assert np.array_equal(s.get_fields(), u32)
        t = torch.from_numpy(u32.astype(np.float32)).cuda()
        s.set_fields(t)
        back = torch.empty_like(t)
        s.get_fields(back)
        torch.cuda.synchronize()
        assert torch.equal(back, t)
        eo = W.energy(m, u32, **kw)
        assert abs(s.energy() - eo) <= 1e-6 * eo
        s.free()


@pytest.mark.parametrize("N", [3, 4, 5, 6, 7])
def test_fp32_meshes_smaller_than_a_tile(N):
    """The FP32 contraction kernels on 1, 2 and 6 elements (one ragged tile, shorter than a
    tile of the field arrays, so every clamped prefetch index lands inside the arrays): the
    right-hand side and one RK step against the oracle, in vacuum and in a medium (N = 7: the
    streamed operator strip)."""
    one_v = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]])
    two_v = np.vstack([one_v, [[0.9, 0.8, 0.95]]])
    cube_v, cube_e = dginputs.kuhn_cube(1, jitter=0.1, permute=True)
    for v, e in ((one_v, np.array([[0, 1, 2, 3]])), (two_v, np.array([[0, 1, 2, 3], [1, 2, 3, 4]])),
                 (cube_v, cube_e)):
        m = Mm.Mesh(v, e, R.ref_element(N))
        u0 = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32")
        eps, mu = dginputs.random_materials(e.shape[0])
        for kw in ({}, dict(eps=eps, mu=mu)):
            say(f"case: N={N} K={e.shape[0]} f32 {'medium' if kw else 'vacuum'}")
            s = P.Solver(v, e, N, "f32", **kw)
            assert rel_l2(gpu_rhs(s, u0), W.rhs(m, u0, **kw)) <= TOL["f32"]
            dt = W.stable_dt(m) / 4
            s.set_fields(u0)
            s.rk_step(dt)
            uo, _ = W.lsrk4_step(m, u0, dt, **kw)
            assert rel_l2(s.get_fields(), uo) <= TOL["f32"]
            s.free()


def test_rhs_rejects_bad_buffers():
    import torch
    v, e, m, u0 = problem(2, 1)
    s = P.Solver(v, e, 2, "f64")
    t = torch.from_numpy(u0).cuda()
    with pytest.raises(P.DGError):
        s.rhs(t, t)          # aliasing input and output
    with pytest.raises(P.DGError):
        s.rhs(t.float(), torch.empty_like(t).float())   # wrong precision

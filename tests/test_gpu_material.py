"""Parity of the heterogeneous-medium and absorbing-face forms of the HIP path with the FP64
oracle (per-element eps and mu: the impedance-weighted upwind flux of Sec. 6; absorbing faces:
zero exterior state). Same tolerances as the vacuum parity tests: relative L2 1e-12 in FP64,
1e-5 in FP32 (the FP32 oracle input is the FP32-rounded field)."""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import gpu_rhs, per_field_rel, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def medium_problem(N, n, seed=21):
    """Jittered, permuted n^3 Kuhn cube; random eps, mu in [1, 4]; absorbing faces on z = 1."""
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    eps, mu = dginputs.random_materials(m.K, seed=seed)
    fb = dginputs.faces_on_plane(v, e, 2, 1.0) * 2
    absorb = dginputs.faces_on_plane(v, m.etov, 2, 1.0).astype(bool)
    u0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    return v, e, m, u0, eps, mu, fb, absorb


@pytest.mark.parametrize("N", range(1, 10))
def test_medium_absorbing_fp64_all_orders(N):
    say(f"case: medium+absorbing N={N} K=48 f64")
    v, e, m, u0, eps, mu, fb, absorb = medium_problem(N, 2)
    s = P.Solver(v, e, N, "f64", face_bc=fb, eps=eps, mu=mu)
    kw = dict(eps=eps, mu=mu, absorb=absorb)
    err = rel_l2(gpu_rhs(s, u0), W.rhs(m, u0, **kw))
    assert err <= TOL["f64"], err
    dt = W.stable_dt(m)
    s.set_fields(u0)
    e0 = s.energy()
    assert abs(e0 - W.energy(m, u0, eps, mu)) <= 1e-12 * e0
    s.solve(dt, 3)
    uo, res = u0, None
    for _ in range(3):
        uo, res = W.lsrk4_step(m, uo, dt, res, **kw)
    assert rel_l2(s.get_fields(), uo) <= TOL["f64"]
    assert s.energy() <= e0 * (1 + 1e-14)


@pytest.mark.parametrize("N,n", [(2, 3), (3, 3), (3, 4), (4, 3), (4, 4), (6, 2)])
def test_medium_absorbing_fp32(N, n):
    """N = 4 runs on the 16-element contraction kernel (K = 162 ragged, 384 full tiles), N = 3
    and N = 6 on 8-element ones, N = 2 on the element-wise kernel; the steady-state loops of the
    contraction kernels at full size are in test_gpu_fullsize.py."""
    say(f"case: medium+absorbing N={N} K={6 * n ** 3} f32")
    v, e, m, u0, eps, mu, fb, absorb = medium_problem(N, n)
    s = P.Solver(v, e, N, "f32", face_bc=fb, eps=eps, mu=mu)
    u32 = rounded(u0, "f32")
    kw = dict(eps=eps, mu=mu, absorb=absorb)
    r = gpu_rhs(s, u32)
    ro = W.rhs(m, u32, **kw)
    err = rel_l2(r, ro)
    say("  rhs rel", err, "per field", per_field_rel(r, ro))
    assert err <= TOL["f32"]
    dt = W.stable_dt(m)
    s.set_fields(u32)
    s.rk_step(dt)
    uo, _ = W.lsrk4_step(m, u32, dt, **kw)
    assert rel_l2(s.get_fields(), uo) <= TOL["f32"]


@pytest.mark.parametrize("prec,N", [("f64", 3), ("f32", 3), ("f32", 4)])
def test_vacuum_with_absorbing_faces(prec, N):
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    fb = dginputs.faces_on_plane(v, e, 0, 0.0) * 2
    absorb = dginputs.faces_on_plane(v, m.etov, 0, 0.0).astype(bool)
    u0 = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), prec)
    s = P.Solver(v, e, N, prec, face_bc=fb)
    assert rel_l2(gpu_rhs(s, u0), W.rhs(m, u0, absorb=absorb)) <= TOL[prec]


def test_uniform_medium_cavity_fp64_twenty_steps():
    eps_v, mu_v = 2.0, 3.0
    v, e = dginputs.kuhn_cube(4)
    m = Mm.Mesh(v, e, R.ref_element(3))
    eps, mu = np.full(m.K, eps_v), np.full(m.K, mu_v)
    u0 = dginputs.cavity_tm110(*m.x, 0.0, eps_v, mu_v)
    s = P.Solver(v, e, 3, "f64", eps=eps, mu=mu)
    dt = W.stable_dt(m)
    s.set_fields(u0)
    e0 = s.energy()
    assert abs(e0 - W.energy(m, u0, eps, mu)) <= 1e-12 * e0
    s.solve(dt, 20)
    uo, res = u0, None
    for _ in range(20):
        uo, res = W.lsrk4_step(m, uo, dt, res, eps=eps, mu=mu)
    assert rel_l2(s.get_fields(), uo) <= TOL["f64"]
    assert s.energy() <= e0 * (1 + 1e-14)


def test_face_conditions_follow_the_given_vertex_order():
    """Elements given with negative orientation: face_bc indexes the faces of etov as given."""
    v, e = dginputs.kuhn_cube(2, jitter=0.1)
    e_user = e.copy()
    flip = np.arange(0, e.shape[0], 3)
    e_user[flip] = e_user[flip][:, [0, 2, 1, 3]]        # negative orientation
    m = Mm.Mesh(v, e_user, R.ref_element(2))
    fb = dginputs.faces_on_plane(v, e_user, 0, 0.0) * 2
    absorb = dginputs.faces_on_plane(v, m.etov, 0, 0.0).astype(bool)
    assert absorb.sum() == (fb == 2).sum() > 0
    assert np.any((fb == 2) != absorb)     # some flipped elements put the face at another index
    u0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    s = P.Solver(v, e_user, 2, "f64", face_bc=fb)
    assert rel_l2(gpu_rhs(s, u0), W.rhs(m, u0, absorb=absorb)) <= TOL["f64"]

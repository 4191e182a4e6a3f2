"""Scattered-field form (incident-field formulation of the scattering example of Sec. 6) on
the GPU against the oracle, through the C ABI.

Scatterer faces on the planes x = 0 and z = 0 (the total field meets a wall there), absorbing
faces on z = 1, walls elsewhere; a plane wave with a linear-plus-sine profile. Every kernel:
FP64 and FP32 at N = 1..7 (element-wise kernel, contraction kernels at FP32 N = 3..7), in
vacuum and in a medium. Checked: the right-hand side at a set time, one RK step from that time
(stage times t + c_i dt), then six more steps through dg_solve (the captured graph advances the
device clock), and the handle's time.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, gpu_rhs, max_rel, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
K_DIR = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
P_POL = np.cross(K_DIR, [1.0, 0.2, 0.1])
P_POL = 0.8 * P_POL / np.linalg.norm(P_POL)
PROFILE = np.array([0.1, -0.4, 0.9, 4.0, 0.3])


def _flags(v, e, etov_oracle):
    f = dginputs.faces_on_plane
    fb = (3 * (f(v, e, 0, 0.0) | f(v, e, 2, 0.0)) + 2 * f(v, e, 2, 1.0)).astype(np.int8)
    scatter = (f(v, etov_oracle, 0, 0.0) | f(v, etov_oracle, 2, 0.0)).astype(bool)
    absorb = f(v, etov_oracle, 2, 1.0).astype(bool)
    return fb, scatter, absorb


def _check(got, want, prec, what):
    err, mx = rel_l2(got, want), max_rel(got, want)
    say(f"  {what}: rel {err:.2e} max {mx:.2e}")
    assert err <= TOL[prec] and mx <= MAX_TOL[prec], what


@pytest.mark.parametrize("medium", [False, True])
@pytest.mark.parametrize("N", range(1, 8))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_scattered_field_matches_oracle(prec, N, medium):
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True, shuffle=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    fb, scatter, absorb = _flags(v, e, m.etov)
    assert scatter.any() and absorb.any()
    kw = dict(scatter=scatter, absorb=absorb, incident=W.PlaneWave(K_DIR, P_POL, PROFILE))
    skw = dict(face_bc=fb)
    if medium:
        eps, mu = dginputs.random_materials(m.K, seed=29)
        kw.update(eps=eps, mu=mu)
        skw.update(eps=eps, mu=mu)
    say(f"case: scattered field N={N} K={m.K} {prec} {'medium' if medium else 'vacuum'}")
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), prec)
    s = P.Solver(v, e, N, prec, **skw)
    s.set_incident(K_DIR, P_POL, PROFILE)
    t0 = 0.37
    s.set_time(t0)
    _check(gpu_rhs(s, u), W.rhs(m, u, t=t0, **kw), prec, "rhs")
    dt = W.stable_dt(m)
    s.set_fields(u)
    s.rk_step(dt)
    uo, res = W.lsrk4_step(m, u, dt, t=t0, **kw)
    _check(s.get_fields(), uo, prec, "1 step")
    s.solve(dt, 4)
    s.solve(dt, 2)
    t = t0 + dt
    for _ in range(6):
        uo, res = W.lsrk4_step(m, uo, dt, res=res, t=t, **kw)
        t += dt
    _check(s.get_fields(), uo, prec, "7 steps")
    assert abs(s.time - t) <= 1e-12 * t
    s.free()


@pytest.mark.parametrize("N,n", [(4, 14), (5, 12)])
def test_scattered_field_steady_state_loop(N, n):
    """A mesh with several tiles per persistent workgroup (FP32 contraction kernels): sampled
    right-hand side and one sampled RK step against the oracle."""
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=True)
    m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
    fb, scatter, absorb = _flags(v, e, m.etov)
    kw = dict(scatter=scatter, absorb=absorb, incident=W.PlaneWave(K_DIR, P_POL, PROFILE))
    say(f"case: scattered field steady state N={N} K={m.K} f32")
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32")
    s = P.Solver(v, e, N, "f32", face_bc=fb)
    s.set_incident(K_DIR, P_POL, PROFILE)
    s.set_time(0.21)
    g = np.random.default_rng(70 + N)
    near = np.nonzero(scatter.any(1))[0]
    sample = np.unique(np.concatenate([g.choice(m.K, 300, replace=False), g.choice(near, 40, replace=False)]))
    r = gpu_rhs(s, u)
    _check(r[:, sample], W.rhs_at(m, u, sample, t=0.21, **kw), "f32", "sampled rhs")
    dt = W.stable_dt(m)
    s.set_fields(u)
    s.rk_step(dt)
    ss = sample[:8]
    _check(s.get_fields()[:, ss], W.lsrk4_step_at(m, u, dt, ss, t=0.21, **kw), "f32", "sampled 1 step")
    s.free()

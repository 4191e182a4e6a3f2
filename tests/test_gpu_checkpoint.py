"""Checkpoint and resume on the GPU: the state of an LSRK4 solve at a step boundary is its
fields and its time (the residual restarts from zero at every step: the first stage's
coefficient is 0), so dg_get_fields + dg_get_time on one handle and dg_set_fields +
dg_set_time on a fresh one resume it exactly. Checked bitwise against the uninterrupted solve,
for the time-dependent scattered-field form (where the restored time matters) and a plain
vacuum solve, in both precisions and on the element-wise and contraction kernels.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import rounded, say

pytestmark = pytest.mark.gpu

K_DIR = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
P_POL = np.cross(K_DIR, [1.0, 0.2, 0.1])
P_POL = 0.8 * P_POL / np.linalg.norm(P_POL)
PROFILE = np.array([0.1, -0.4, 0.9, 4.0, 0.3])


@pytest.mark.parametrize("scattered", [False, True])
@pytest.mark.parametrize("prec,N", [("f64", 2), ("f64", 3), ("f32", 4), ("f32", 6)])
def test_solve_2n_equals_solve_n_save_load_solve_n(prec, N, scattered):
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True)
    skw = {}
    if scattered:
        f = dginputs.faces_on_plane
        skw["face_bc"] = (3 * f(v, e, 0, 0.0) + 2 * f(v, e, 2, 1.0)).astype(np.int8)
    say(f"case: checkpoint N={N} {prec} {'scattered field' if scattered else 'vacuum'}")

    def fresh():
        s = P.Solver(v, e, N, prec, **skw)
        if scattered:
            s.set_incident(K_DIR, P_POL, PROFILE)
        return s

    a = fresh()
    x = a.nodes()
    u0 = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *x), prec)
    dt = a.stable_dt(0.5)
    t0 = 0.25
    a.set_fields(u0)
    a.set_time(t0)
    a.solve(dt, 10)                       # uninterrupted: 2n steps
    full = a.get_fields()

    b = fresh()
    b.set_fields(u0)
    b.set_time(t0)
    b.solve(dt, 5)                        # n steps, then save
    saved_u, saved_t = b.get_fields(), b.time
    b.free()
    c = fresh()                           # load into a new handle, n more steps
    c.set_fields(saved_u)
    c.set_time(saved_t)
    c.solve(dt, 5)
    assert np.array_equal(c.get_fields(), full)
    assert c.time == a.time
    a.free()
    c.free()

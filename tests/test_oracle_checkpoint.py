"""Checkpoint and resume on the oracle: 2n LSRK4 steps equal n steps, a restart from the saved
fields and time with the residual reset, and n more steps, bitwise; also for the scattered-field
form, whose operator depends on the time."""
import numpy as np

import dginputs
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R


def _run(m, u, dt, n, t0, kw, res=None):
    t = t0
    for _ in range(n):
        u, res = W.lsrk4_step(m, u, dt, res=res, t=t, **kw)
        t += dt
    return u, res, t


def test_solve_2n_equals_solve_n_save_load_solve_n():
    v, e = dginputs.kuhn_cube(2, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(3))
    u0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    dt = W.stable_dt(m)
    f = dginputs.faces_on_plane
    scatter = f(v, m.etov, 0, 0.0).astype(bool)
    inc = W.PlaneWave(np.array([0.0, 0.6, 0.8]), np.array([1.0, 0.0, 0.0]), np.array([0.1, -0.4, 0.9, 4.0, 0.3]))
    for kw in ({}, dict(scatter=scatter, incident=inc)):
        full, _, t_full = _run(m, u0, dt, 6, 0.3, kw)
        half, res, t_half = _run(m, u0, dt, 3, 0.3, kw)
        assert np.any(res != 0.0)                      # the dropped residual is not trivial
        resumed, _, t_end = _run(m, half, dt, 3, t_half, kw)
        assert np.array_equal(resumed, full) and t_end == t_full

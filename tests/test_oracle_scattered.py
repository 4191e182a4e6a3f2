"""Pins of the oracle's scattered-field form (the incident-field formulation of the scattering
example of Sec. 6): on a scatterer face the total field u_s + u_inc meets the perfectly
conducting wall.

- a linear plane wave is reproduced exactly by the DG operator (it is a polynomial of degree
  one in space, continuous across faces, and solves Maxwell's equations), so the scattered-field
  solution must equal the total-field solution of the walled cavity minus the interpolated
  incident wave, step by step, to rounding: this fixes the factor 2, the sign, that only E
  enters, and the stage times c_i of the Runge-Kutta method (the incident wave varies in t);
- with a sinusoidal incident wave the exact scattered field of the walled unit cube is the
  (1,1,0) cavity mode minus the incident wave, and the oracle converges to it under h-refinement;
- a scatterer face without incident wave is a perfectly conducting wall (bitwise).
"""
import math

import numpy as np
import pytest

import dginputs
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R


def _unit(v):
    v = np.asarray(v, dtype=np.float64)
    return v / np.linalg.norm(v)


K_DIR = _unit([0.3, -0.5, 0.8])
P_POL = _unit(np.cross(K_DIR, [1.0, 0.2, 0.1]))


def _plane_wave_closed_form(x, y, z, t, c):
    """E = p f(k.x - t), H = (k x p) f(k.x - t), and their time derivatives, written out from
    the plane-wave solution of Maxwell's equations in vacuum (profile f(s) = c0 + c1 s +
    c2 sin(c3 s + c4))."""
    s = K_DIR[0] * x + K_DIR[1] * y + K_DIR[2] * z - t
    f = c[0] + c[1] * s + c[2] * np.sin(c[3] * s + c[4])
    fp = c[1] + c[2] * c[3] * np.cos(c[3] * s + c[4])
    h = np.cross(K_DIR, P_POL)
    u = np.stack([P_POL[i] * f for i in range(3)] + [h[i] * f for i in range(3)])
    dudt = -np.stack([P_POL[i] * fp for i in range(3)] + [h[i] * fp for i in range(3)])
    return u, dudt


def _walled_mesh(N, n, jitter=0.15):
    v, e = dginputs.kuhn_cube(n, jitter=jitter, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    return m


def test_plane_wave_solves_maxwell():
    """The oracle's incident field is the closed-form plane wave, and it solves Maxwell's
    equations: finite differences in space and time."""
    c = np.array([0.2, -0.7, 1.3, 2.1, 0.4])
    pw = W.PlaneWave(K_DIR, P_POL, c)
    g = np.random.default_rng(5)
    x, y, z = g.uniform(0, 1, (3, 40))
    t = 0.37
    u, dudt = _plane_wave_closed_form(x, y, z, t, c)
    assert np.max(np.abs(pw.fields(x, y, z, t) - u)) < 1e-14
    h = 1e-5
    def d(axis):
        dx = np.zeros(3)
        dx[axis] = h
        return (pw.fields(x + dx[0], y + dx[1], z + dx[2], t) - pw.fields(x - dx[0], y - dx[1], z - dx[2], t)) / (2 * h)
    dX, dY, dZ = d(0), d(1), d(2)
    curlH = np.stack([dY[5] - dZ[4], dZ[3] - dX[5], dX[4] - dY[3]])
    curlE = np.stack([dY[2] - dZ[1], dZ[0] - dX[2], dX[1] - dY[0]])
    dt = (pw.fields(x, y, z, t + h) - pw.fields(x, y, z, t - h)) / (2 * h)
    assert np.max(np.abs(dt[:3] - curlH)) < 1e-8
    assert np.max(np.abs(dt[3:] + curlE)) < 1e-8


@pytest.mark.parametrize("N", [1, 2, 3])
def test_linear_incident_wave_reproduces_total_field_exactly(N):
    """Scattered field = total field of the walled cavity - interpolated incident wave, for the
    right-hand side and for three RK steps (all walls are scatterer faces)."""
    m = _walled_mesh(N, 2)
    c = np.array([0.4, -1.3, 0.0, 0.0, 0.0])      # f(s) = 0.4 - 1.3 s: linear in x and t
    pw = W.PlaneWave(K_DIR, P_POL, c)
    scatter = m.boundary.copy()
    x, y, z = m.x
    u_tot0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x, y, z)
    t0 = 0.3
    inc0, dinc0 = _plane_wave_closed_form(x, y, z, t0, c)
    # right-hand side: L_scat(u_s, t) = L_wall(u_s + u_inc(t)) - d/dt u_inc(t)
    us0 = u_tot0 - inc0
    r_s = W.rhs(m, us0, scatter=scatter, incident=pw, t=t0)
    r_t = W.rhs(m, u_tot0)
    scale = np.linalg.norm(r_t)
    assert np.linalg.norm(r_s - (r_t - dinc0)) <= 1e-12 * scale
    # three steps
    dt = W.stable_dt(m)
    ut, us, t = u_tot0, us0, t0
    rt = rs = None
    for _ in range(3):
        ut, rt = W.lsrk4_step(m, ut, dt, res=rt)
        us, rs = W.lsrk4_step(m, us, dt, res=rs, t=t, scatter=scatter, incident=pw)
        t += dt
    inc, _ = _plane_wave_closed_form(x, y, z, t, c)
    assert np.linalg.norm(us - (ut - inc)) <= 1e-12 * np.linalg.norm(ut)
    # the incident wave matters
    assert np.linalg.norm(inc - _plane_wave_closed_form(x, y, z, t0, c)[0]) > 1e-3 * np.linalg.norm(inc)


def test_scatterer_without_incident_wave_is_a_wall():
    m = _walled_mesh(3, 2)
    u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    zero = W.PlaneWave(K_DIR, P_POL, np.zeros(5))
    a = W.rhs(m, u)
    assert np.array_equal(W.rhs(m, u, scatter=m.boundary, incident=zero, t=0.7), a)
    assert np.array_equal(W.rhs(m, u, scatter=m.boundary, incident=None), a)


def test_sampled_forms_match_with_scatterers():
    m = _walled_mesh(2, 3)
    u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    pw = W.PlaneWave(K_DIR, P_POL, np.array([0.1, 0.3, 0.8, 3.0, 0.2]))
    sc = m.boundary & (m.x[2].reshape(m.K, -1).mean(1) < 0.5)[:, None]
    ab = m.boundary & ~sc
    kw = dict(scatter=sc, absorb=ab, incident=pw)
    elems = np.array([0, 5, 17, m.K - 1])
    assert np.array_equal(W.rhs_at(m, u, elems, t=0.4, **kw), W.rhs(m, u, t=0.4, **kw)[:, elems])
    dt = W.stable_dt(m)
    full, _ = W.lsrk4_step(m, u, dt, t=0.4, **kw)
    assert np.allclose(W.lsrk4_step_at(m, u, dt, elems, t=0.4, **kw), full[:, elems], rtol=0, atol=1e-14)


def _scattered_error(N, n, T):
    """Relative L2 error at time T of the scattered field of the walled unit cube lit by a
    sinusoidal plane wave, against the exact scattered field (cavity mode minus incident)."""
    m = _walled_mesh(N, n)
    c = np.array([0.0, 0.0, 0.7, 2.5, 0.3])
    pw = W.PlaneWave(K_DIR, P_POL, c)
    x, y, z = m.x
    us = dginputs.cavity_tm110(x, y, z, 0.0) - _plane_wave_closed_form(x, y, z, 0.0, c)[0]
    nsteps = int(math.ceil(T / W.stable_dt(m)))
    dt = T / nsteps
    res, t = None, 0.0
    for _ in range(nsteps):
        us, res = W.lsrk4_step(m, us, dt, res=res, t=t, scatter=m.boundary, incident=pw)
        t += dt
    exact = dginputs.cavity_tm110(x, y, z, T) - _plane_wave_closed_form(x, y, z, T, c)[0]
    err, ref = W.l2_error(m, us, exact)
    return err / ref


@pytest.mark.slow
@pytest.mark.parametrize("N", [1, 2])
def test_sinusoidal_incident_wave_converges_to_exact_scattered_field(N):
    errs = [_scattered_error(N, n, 0.25) for n in (2, 4)]
    rate = math.log(errs[0] / errs[1]) / math.log(2.0)
    assert errs[1] < (0.1 if N == 1 else 0.01)
    assert rate >= N + 0.5, (errs, rate)


def _identity_mismatch(N=2):
    """Relative mismatch of the exact identity above after two RK steps."""
    m = _walled_mesh(N, 2)
    c = np.array([0.4, -1.3, 0.0, 0.0, 0.0])
    pw = W.PlaneWave(K_DIR, P_POL, c)
    x, y, z = m.x
    ut = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x, y, z)
    t = 0.3
    us = ut - _plane_wave_closed_form(x, y, z, t, c)[0]
    dt = W.stable_dt(m)
    rt = rs = None
    for _ in range(2):
        ut, rt = W.lsrk4_step(m, ut, dt, res=rt)
        us, rs = W.lsrk4_step(m, us, dt, res=rs, t=t, scatter=m.boundary, incident=pw)
        t += dt
    return np.linalg.norm(us - (ut - _plane_wave_closed_form(x, y, z, t, c)[0])) / np.linalg.norm(ut)


ORIG_INC = W._incident_at_faces


@pytest.mark.parametrize("name,patch", [
    ("incident E counted once instead of twice", lambda mp: mp.setattr(
        W, "_incident_at_faces", lambda *a: None if ORIG_INC(*a) is None else 0.5 * ORIG_INC(*a))),
    ("incident E with the wrong sign", lambda mp: mp.setattr(
        W, "_incident_at_faces", lambda *a: None if ORIG_INC(*a) is None else -ORIG_INC(*a))),
    ("stages evaluated at the step's start time", lambda mp: mp.setattr(W, "RK4C", np.zeros(5))),
    ("stages evaluated at the step's end time", lambda mp: mp.setattr(W, "RK4C", np.ones(5))),
])
def test_planted_scattered_field_mistakes_are_caught(monkeypatch, name, patch):
    assert _identity_mismatch() < 1e-12
    patch(monkeypatch)
    assert _identity_mismatch() > 1e-6, name

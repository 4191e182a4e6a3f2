"""Pins of the oracle's discrete energy and L2 norm against closed forms (CPU only).

The discrete energy is 1/2 sum_k J_k (eps u_E^T M u_E + mu u_H^T M u_H) and the L2 norm is
sqrt(sum_k J_k u^T M u) (the energy of Sec. 6's stability remark and the L2 error of Sec. 6's
convergence table; M is the reference mass matrix of eq. dg-global-matrices). Both are pinned
to values that do not come from the oracle:

- exact: for constant fields the nodal interpolant is exact and M integrates it exactly, so
  the norm of the constant 1 in all six fields over the unit cube is sqrt(6) and the energy
  is 1/2 (3 eps + 3 mu), on any mesh of the cube (jittering moves interior vertices only);
- closed form with h-convergence: the (1,1,0) TM mode of the unit-cube cavity in a uniform
  medium (eps = 2, mu = 3) has energy eps/8 at t = 0 (all electric, 1/2 eps int E_z^2) and
  the same total at a quarter period (all magnetic, 1/2 mu int |H|^2); its L2 norm is 1/2 at
  t = 0 and sqrt(eps/mu)/2 at a quarter period. On jittered meshes (non-uniform J) the
  discrete values converge to these at the interpolation order.

A missing 1/2, a missing or misplaced J_k, or exchanged eps / mu weights each fail one of
these (checked by planted mistakes in test_oracle_mutations.py).
"""
import math

import numpy as np
import pytest

import dginputs
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

EPS, MU = 2.0, 3.0


def jittered_mesh(n, N):
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
    return Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)


def quarter_period():
    return (math.pi / 2.0) / (math.pi * math.sqrt(2.0) / math.sqrt(EPS * MU))


def energy_pins_hold(energy_fn, l2_fn, rtol=1e-12):
    """True when the exact constant-field pins and the cavity closed forms (with
    h-convergence) hold for the given energy and norm functions."""
    ok = True
    m = jittered_mesh(2, 2)
    assert np.ptp(m.J) > 0.05 * np.mean(m.J)          # the Jacobians really differ
    eps, mu = np.full(m.K, EPS), np.full(m.K, MU)
    ones = np.ones((6, m.K, m.ref.Np))
    ok &= abs(energy_fn(m, ones, eps, mu) - 0.5 * (3 * EPS + 3 * MU)) <= rtol * 7.5
    ok &= abs(energy_fn(m, ones, None, None) - 3.0) <= rtol * 3.0
    ok &= abs(l2_fn(m, ones, np.zeros_like(ones))[0] - math.sqrt(6.0)) <= rtol * 3.0
    # only the E fields set: eps weights them; only the H fields: mu weights them
    half = ones.copy()
    half[3:] = 0.0
    ok &= abs(energy_fn(m, half, eps, mu) - 1.5 * EPS) <= rtol * 3.0
    half = ones.copy()
    half[:3] = 0.0
    ok &= abs(energy_fn(m, half, eps, mu) - 1.5 * MU) <= rtol * 4.5
    # cavity mode: convergence to the closed form at t = 0 and a quarter period
    tq = quarter_period()
    for t, e_exact, n_exact in ((0.0, EPS / 8.0, 0.5), (tq, EPS / 8.0, 0.5 * math.sqrt(EPS / MU))):
        errs_e, errs_n = [], []
        for n in (2, 4):
            m = jittered_mesh(n, 4)
            eps, mu = np.full(m.K, EPS), np.full(m.K, MU)
            u = dginputs.cavity_tm110(*m.x, t, EPS, MU)
            errs_e.append(abs(energy_fn(m, u, eps, mu) - e_exact) / e_exact)
            errs_n.append(abs(l2_fn(m, u, np.zeros_like(u))[0] - n_exact) / n_exact)
        # interpolation error at N = 4: halving h divides the error by far more than 10
        ok &= errs_e[1] <= 5e-5 and errs_e[1] <= errs_e[0] / 10.0
        ok &= errs_n[1] <= 5e-5 and errs_n[1] <= errs_n[0] / 10.0
    return bool(ok)


def test_energy_and_norm_match_closed_forms():
    assert energy_pins_hold(W.energy, W.l2_error)


def test_cavity_energy_is_conserved_between_electric_and_magnetic():
    """At t = 0 the energy is all electric and at a quarter period all magnetic; the discrete
    values at the two times agree to the interpolation error."""
    m = jittered_mesh(4, 4)
    eps, mu = np.full(m.K, EPS), np.full(m.K, MU)
    u0 = dginputs.cavity_tm110(*m.x, 0.0, EPS, MU)
    uq = dginputs.cavity_tm110(*m.x, quarter_period(), EPS, MU)
    assert np.max(np.abs(u0[3:])) == 0.0 and np.max(np.abs(uq[:3])) < 1e-15
    e0, eq = W.energy(m, u0, eps, mu), W.energy(m, uq, eps, mu)
    assert abs(e0 - eq) <= 1e-5 * e0 and abs(e0 - EPS / 8.0) <= 3e-5 * e0


@pytest.mark.parametrize("N", [1, 4, 7])
def test_norm_of_a_difference(N):
    """l2_error(u, v) is (||u - v||, ||v||): the norm of a constant difference c over the unit
    cube is |c| sqrt(6) whatever v is."""
    m = jittered_mesh(1, N)
    g = np.random.default_rng(5)
    v = g.standard_normal((6, m.K, m.ref.Np))
    err, nrm = W.l2_error(m, v + 0.25, v)
    assert abs(err - 0.25 * math.sqrt(6.0)) <= 1e-12
    assert abs(nrm - W.l2_error(m, v, np.zeros_like(v))[0]) <= 1e-14 * nrm

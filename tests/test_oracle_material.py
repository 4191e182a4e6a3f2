"""Pins of the oracle's heterogeneous-medium and absorbing-boundary forms (Sec. 6: the
impedance-weighted upwind flux, Z = sqrt(mu/eps), Y = 1/Z; the characteristic absorbing
condition named for the scattering example, read as a zero exterior state).

- two-tetrahedron brute force with per-element eps, mu and an absorbing face: independent
  weak-form assembly equals the oracle operator;
- energy: with the eps/mu-weighted mass, the upwind operator is dissipative (with absorbing
  faces too) and the central one with walls only is skew;
- an absorbing face is transparent to an outgoing plane wave and stops an incoming one;
- a uniform medium scales the cavity mode by the wave speed and impedance: the oracle's
  right-hand side matches the closed form's time derivative and the error falls with h.
"""
import math

import numpy as np
import pytest

import dginputs
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

from test_oracle_maxwell import assemble, brute_force_operator, mass_weight


def weighted_mass(mesh, eps, mu):
    Mw = mass_weight(mesh)
    w = np.concatenate([np.repeat(eps, mesh.ref.Np)] * 3 + [np.repeat(mu, mesh.ref.Np)] * 3)
    return Mw * w[:, None]


@pytest.mark.parametrize("N", [1, 2])
def test_two_tet_brute_force_with_materials_and_absorbing_face(N):
    vxyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.05, 0.9, 0.1], [0.1, 0.0, 1.1],
                     [0.9, 0.8, 0.95]])
    etov = Mm.orient(vxyz, np.array([[0, 1, 2, 3], [1, 2, 3, 4]]))
    eps = np.array([2.0, 1.3])
    mu = np.array([1.5, 3.0])
    mo = Mm.Mesh(vxyz, etov, R.ref_element(N))
    absorb = np.zeros((2, 4), dtype=bool)
    bf = np.argwhere(mo.boundary)
    absorb[tuple(bf[0])] = True          # one wall of each element absorbs
    absorb[tuple(bf[-1])] = True
    A_bf, _ = brute_force_operator(vxyz, etov, N, eps=eps, mu=mu, absorb=absorb)
    A = assemble(mo, eps=eps, mu=mu, absorb=absorb)
    assert np.linalg.norm(A - A_bf) <= 1e-11 * np.linalg.norm(A)
    # the material and the absorbing face both matter
    assert np.linalg.norm(A - assemble(mo)) > 1e-2 * np.linalg.norm(A)
    assert np.linalg.norm(A - assemble(mo, eps=eps, mu=mu)) > 1e-3 * np.linalg.norm(A)


@pytest.mark.parametrize("N", [1, 2])
def test_weighted_energy_dissipative_and_skew(N):
    v, e = dginputs.kuhn_cube(1, jitter=0.0)
    m = Mm.Mesh(v, e, R.ref_element(N))
    eps, mu = dginputs.random_materials(m.K, seed=11)
    Mw = weighted_mass(m, eps, mu)
    absorb = dginputs.faces_on_plane(v, e, 2, 1.0).astype(bool)
    assert absorb.any()
    for kw in ({}, {"absorb": absorb}):
        A = assemble(m, eps=eps, mu=mu, **kw)
        S = Mw @ A + A.T @ Mw
        scale = np.linalg.norm(Mw @ A)
        assert np.max(np.linalg.eigvalsh(S)) <= 1e-12 * scale
    Ac = assemble(m, alpha=0.0, eps=eps, mu=mu)
    assert np.linalg.norm(Mw @ Ac + Ac.T @ Mw) <= 1e-12 * np.linalg.norm(Mw @ Ac)
    # with the plain (unweighted) mass the central operator is not skew: the weights matter
    Mu = mass_weight(m)
    assert np.linalg.norm(Mu @ Ac + Ac.T @ Mu) > 1e-3 * np.linalg.norm(Mu @ Ac)


def test_absorbing_face_passes_outgoing_and_blocks_incoming_plane_waves():
    v, e = dginputs.kuhn_cube(1)
    m = Mm.Mesh(v, e, R.ref_element(2))
    absorb = dginputs.faces_on_plane(v, e, 2, 1.0).astype(bool)     # outward normal +z
    eps = np.full(m.K, 2.0)
    mu = np.full(m.K, 0.5)
    Z = math.sqrt(0.5 / 2.0)
    ex = np.array([0.3, -1.1, 0.0])                # tangential to the face
    h_out = np.cross([0.0, 0.0, 1.0], ex) / Z      # E x H along +n: leaves the domain
    for h, outgoing in ((h_out, True), (-h_out, False)):
        u = np.zeros((6, m.K, m.ref.Np))
        u[:3] = ex[:, None, None]
        u[3:] = h[:, None, None]
        flux = W.surface_flux(m, u, eps=eps, mu=mu, absorb=absorb)     # 6, K, 4, Nfp
        on = flux[:, absorb]
        if outgoing:
            assert np.max(np.abs(on)) <= 1e-14
        else:
            # incoming wave: the flux is the full jump n x (Z+ [H] - n x [E]) / (Z- + Z+)
            assert np.max(np.abs(on)) > 0.5


def test_uniform_medium_cavity_rhs_is_the_closed_form_time_derivative():
    eps, mu = 2.0, 3.0
    errs = []
    for n in (2, 4):
        v, e = dginputs.kuhn_cube(n)
        m = Mm.Mesh(v, e, R.ref_element(3))
        x, y, z = m.x
        w = math.pi * math.sqrt(2.0) / math.sqrt(eps * mu)
        u0 = dginputs.cavity_tm110(x, y, z, 0.0, eps, mu)
        # d/dt at t = 0: E' = 0, H' = w * (H at t = pi / (2 w))
        dudt = w * dginputs.cavity_tm110(x, y, z, math.pi / (2 * w), eps, mu)
        dudt[:3] = 0.0
        r = W.rhs(m, u0, eps=np.full(m.K, eps), mu=np.full(m.K, mu))
        err, nrm = W.l2_error(m, r, dudt)
        errs.append(err / nrm)
        # the vacuum operator is wrong for this medium by an O(1) amount
        err_vac, _ = W.l2_error(m, W.rhs(m, u0), dudt)
        assert err_vac / nrm > 0.3
    assert errs[1] < errs[0] / 6.0


@pytest.mark.slow
def test_uniform_medium_cavity_converges():
    eps, mu, N, T = 2.0, 3.0, 2, 0.5
    errs = []
    for n in (1, 2, 4):
        v, e = dginputs.kuhn_cube(n)
        m = Mm.Mesh(v, e, R.ref_element(N))
        x, y, z = m.x
        u = dginputs.cavity_tm110(x, y, z, 0.0, eps, mu)
        ns = int(math.ceil(T / W.stable_dt(m)))
        dt = T / ns
        res = None
        kw = dict(eps=np.full(m.K, eps), mu=np.full(m.K, mu))
        for _ in range(ns):
            u, res = W.lsrk4_step(m, u, dt, res, **kw)
        err, _ = W.l2_error(m, u, dginputs.cavity_tm110(x, y, z, T, eps, mu))
        errs.append(err)
    rate = math.log(errs[-2] / errs[-1]) / math.log(2.0)
    assert rate >= N + 0.5


def test_sampled_rhs_and_step_equal_the_full_ones_in_a_medium():
    """The sampled forms (used at full mesh sizes) with per-element eps, mu and absorbing faces
    equal the full right-hand side and step bitwise at the sampled elements."""
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True, shuffle=True)
    m = Mm.Mesh(v, e, R.ref_element(3))
    eps, mu = dginputs.random_materials(m.K, seed=21)
    absorb = dginputs.faces_on_plane(v, m.etov, 2, 1.0).astype(bool)
    assert absorb.any()
    kw = dict(eps=eps, mu=mu, absorb=absorb)
    u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    idx = np.unique(np.concatenate([np.nonzero(absorb.any(1))[0][:3], [0, 7, 50, m.K - 1]]))
    assert np.array_equal(W.rhs_at(m, u, idx, **kw), W.rhs(m, u, **kw)[:, idx])
    dt = W.stable_dt(m)
    full, _ = W.lsrk4_step(m, u, dt, **kw)
    assert np.array_equal(W.lsrk4_step_at(m, u, dt, idx, **kw), full[:, idx])

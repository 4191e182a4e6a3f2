"""Planted mistakes in the oracle (CPU only): each must be caught by a pin.

Each mutation patches one piece of the oracle for the duration of a test and shows that the
two-tetrahedron brute force (or the energy pin) no longer agrees with it.
"""
import numpy as np
import pytest

from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

from test_oracle_maxwell import assemble, brute_force_operator, mass_weight

VXYZ = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.05, 0.9, 0.1], [0.1, 0.0, 1.1],
                 [0.9, 0.8, 0.95]])
ETOV = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
N = 2


@pytest.fixture(scope="module")
def reference_operator():
    A_bf, _ = brute_force_operator(VXYZ, Mm.orient(VXYZ, ETOV), N)
    return A_bf


def _mismatch(A_bf):
    mo = Mm.Mesh(VXYZ, ETOV, R.ref_element(N))
    A = assemble(mo)
    return np.linalg.norm(A - A_bf) / np.linalg.norm(A_bf)


def test_unmutated_oracle_agrees(reference_operator):
    assert _mismatch(reference_operator) < 1e-11


def _swap_eh_volume(mesh, u):
    v = ORIG_VOLUME(mesh, u)
    return np.concatenate([-v[3:], -v[:3]])


ORIG_VOLUME = W.volume_term
ORIG_FLUX = W.surface_flux


def _flux_wrong_normal(mesh, u, *args, **kw):
    saved = mesh.n
    mesh.n = -saved
    try:
        return ORIG_FLUX(mesh, u, *args, **kw)
    finally:
        mesh.n = saved


def _flux_no_neighbour(mesh, u, *args, **kw):
    saved = mesh.vmapP
    mesh.vmapP = mesh.vmapM
    try:
        return ORIG_FLUX(mesh, u, *args, **kw)
    finally:
        mesh.vmapP = saved


def _flux_half(mesh, u, *args, **kw):
    return 0.5 * ORIG_FLUX(mesh, u, *args, **kw)


@pytest.mark.parametrize("name,target,replacement", [
    ("E/H blocks exchanged in the volume term", "volume_term", _swap_eh_volume),
    ("normal sign flipped in the flux", "surface_flux", _flux_wrong_normal),
    ("neighbour trace replaced by own trace", "surface_flux", _flux_no_neighbour),
    ("flux scaled by 1/2 twice", "surface_flux", _flux_half),
])
def test_planted_rhs_mistake_is_caught(monkeypatch, reference_operator, name, target, replacement):
    monkeypatch.setattr(W, target, replacement)
    assert _mismatch(reference_operator) > 1e-3, name


def test_transposed_derivative_matrix_is_caught(monkeypatch, reference_operator):
    ref = R.ref_element(N)
    monkeypatch.setattr(ref, "Dr", ref.Dr.T.copy())
    assert _mismatch(reference_operator) > 1e-3


def test_lift_without_face_mass_is_caught(monkeypatch, reference_operator):
    ref = R.ref_element(N)
    monkeypatch.setattr(ref, "LIFT", np.linalg.solve(ref.M, (ref.Emat != 0).astype(float)))
    assert _mismatch(reference_operator) > 1e-3


def test_anti_dissipative_flux_is_caught():
    v = VXYZ
    m = Mm.Mesh(v, ETOV, R.ref_element(N))
    A = assemble(m, alpha=-1.0)
    Mw = mass_weight(m)
    S = Mw @ A + A.T @ Mw
    assert np.max(np.linalg.eigvalsh(S)) > 1e-6 * np.linalg.norm(Mw @ A)


# ---------------------------------------------------------------------------------------
# heterogeneous medium and absorbing faces

EPS = np.array([2.0, 1.3])
MU = np.array([1.5, 3.0])


def _material_case():
    etov = Mm.orient(VXYZ, ETOV)
    mo = Mm.Mesh(VXYZ, etov, R.ref_element(N))
    absorb = np.zeros((2, 4), dtype=bool)
    bf = np.argwhere(mo.boundary)
    absorb[tuple(bf[0])] = True
    absorb[tuple(bf[-1])] = True
    A_bf, _ = brute_force_operator(VXYZ, etov, N, eps=EPS, mu=MU, absorb=absorb)
    return mo, absorb, A_bf


ORIG_IMP = W._impedances
ORIG_ASSEMBLE = W._assemble


def _impedances_swapped(mesh, elems, eps, mu):
    zm, zp, ym, yp = ORIG_IMP(mesh, elems, eps, mu)
    return zp, zm, yp, ym


def _assemble_without_mu(ref, vol, flux, Fscale, eps_k, mu_k):
    return ORIG_ASSEMBLE(ref, vol, flux, Fscale, eps_k, None)


@pytest.mark.parametrize("name,target,replacement", [
    ("interior and exterior impedances exchanged", "_impedances", _impedances_swapped),
    ("absorbing faces treated as walls", "_check_absorb", lambda mesh, absorb: None),
    ("H rows not divided by mu", "_assemble", _assemble_without_mu),
])
def test_planted_material_mistake_is_caught(monkeypatch, name, target, replacement):
    mo, absorb, A_bf = _material_case()
    assert np.linalg.norm(assemble(mo, eps=EPS, mu=MU, absorb=absorb) - A_bf) < 1e-11 * np.linalg.norm(A_bf)
    monkeypatch.setattr(W, target, replacement)
    A = assemble(mo, eps=EPS, mu=MU, absorb=absorb)
    assert np.linalg.norm(A - A_bf) > 1e-3 * np.linalg.norm(A_bf), name


# ---------------------------------------------------------------------------------------
# discrete energy and L2 norm

from test_oracle_energy import energy_pins_hold  # noqa: E402


def _energy_without_half(mesh, u, eps=None, mu=None):
    return 2.0 * W.energy(mesh, u, eps, mu)


def _energy_without_J(mesh, u, eps=None, mu=None):
    saved = mesh.J
    mesh.J = np.ones_like(saved)
    try:
        return W.energy(mesh, u, eps, mu)
    finally:
        mesh.J = saved


def _energy_eps_mu_exchanged(mesh, u, eps=None, mu=None):
    return W.energy(mesh, u, mu, eps)


def _norm_without_J(mesh, u, uref):
    saved = mesh.J
    mesh.J = np.ones_like(saved)
    try:
        return W.l2_error(mesh, u, uref)
    finally:
        mesh.J = saved


def _norm_squared(mesh, u, uref):
    a, b = W.l2_error(mesh, u, uref)
    return a * a, b * b


def test_unmutated_energy_and_norm_hold():
    assert energy_pins_hold(W.energy, W.l2_error)


@pytest.mark.parametrize("name,energy_fn,l2_fn", [
    ("energy without the factor 1/2", _energy_without_half, W.l2_error),
    ("energy without the Jacobian", _energy_without_J, W.l2_error),
    ("eps and mu weights exchanged", _energy_eps_mu_exchanged, W.l2_error),
    ("norm without the Jacobian", W.energy, _norm_without_J),
    ("norm squared instead of its root", W.energy, _norm_squared),
])
def test_planted_energy_or_norm_mistake_is_caught(name, energy_fn, l2_fn):
    assert not energy_pins_hold(energy_fn, l2_fn), name

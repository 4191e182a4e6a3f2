"""Pins of the oracle's reference element against what mathematics and the paper fix.

Each test names the fact it checks; none re-types the oracle's formulas.
"""
import itertools
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import refelem as R


def tet_quadrature(q):
    """Collapsed (Stroud) rule on the reference tetrahedron, exact to degree 2q-1 (test helper):
    Gauss-Legendre in a, Gauss-Jacobi(1,0) in b, Gauss-Jacobi(2,0) in c."""
    xa, wa = np.polynomial.legendre.leggauss(q)
    xb, wb = R.gauss_jacobi(1.0, 0.0, q)
    xc, wc = R.gauss_jacobi(2.0, 0.0, q)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    W = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]) / 8.0
    r = (1 + A) * (1 - B) * (1 - C) / 4 - 1
    s = (1 + B) * (1 - C) / 2 - 1
    t = C
    return np.stack([r.ravel(), s.ravel(), t.ravel()], axis=1), W.ravel()


def tri_quadrature(q):
    """Collapsed rule on the reference triangle (-1,-1),(1,-1),(-1,1), degree 2q-1."""
    xa, wa = np.polynomial.legendre.leggauss(q)
    xb, wb = R.gauss_jacobi(1.0, 0.0, q)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = wa[:, None] * wb[None, :] / 2.0
    r = (1 + A) * (1 - B) / 2 - 1
    s = B
    return np.stack([r.ravel(), s.ravel()], axis=1), W.ravel()


def lagrange_at(ref, pts):
    """Values of the nodal Lagrange basis at points, via the basis expansion (Np points x Np)."""
    Vq = R.vandermonde3d(ref.N, pts)
    return Vq @ np.linalg.inv(ref.V)


def test_dof_counts_match_paper_table():
    for N, Np, Nfp, NfNfp in read_golden("dof_counts.txt"):
        ref = R.ref_element(int(N))
        assert ref.Np == int(Np)
        assert ref.Nfp == int(Nfp)
        assert ref.LIFT.shape == (int(Np), int(NfNfp))
        assert ref.Fmask.shape == (4, int(Nfp))


@pytest.mark.parametrize("alpha,beta", [(0, 0), (1, 0), (2, 0), (5, 0), (1, 1), (3, 2)])
def test_jacobi_orthonormal_under_weight(alpha, beta):
    # Gauss-Legendre quadrature of the weighted product, independent of Golub-Welsch.
    x, w = np.polynomial.legendre.leggauss(40)
    wt = (1 - x) ** alpha * (1 + x) ** beta
    P = np.stack([R.jacobi_normalized(x, alpha, beta, n) for n in range(7)])
    G = (P * wt * w) @ P.T
    assert np.max(np.abs(G - np.eye(7))) < 1e-12


def test_jacobi_derivative_matches_difference_quotient():
    x = np.linspace(-0.9, 0.9, 11)
    h = 1e-6
    for n in range(1, 7):
        fd = (R.jacobi_normalized(x + h, 2, 0, n) - R.jacobi_normalized(x - h, 2, 0, n)) / (2 * h)
        assert np.max(np.abs(fd - R.jacobi_normalized_deriv(x, 2, 0, n))) < 1e-6


def test_gll_points_closed_forms():
    assert np.allclose(R.gll_points(2), [-1, 0, 1], atol=1e-15)
    assert np.allclose(R.gll_points(3), [-1, -1 / math.sqrt(5), 1 / math.sqrt(5), 1], atol=1e-15)
    a = math.sqrt(3.0 / 7.0)
    assert np.allclose(R.gll_points(4), [-1, -a, 0, a, 1], atol=1e-15)
    b = math.sqrt(1.0 / 3.0 - 2.0 * math.sqrt(7.0) / 21.0)
    c = math.sqrt(1.0 / 3.0 + 2.0 * math.sqrt(7.0) / 21.0)
    assert np.allclose(R.gll_points(5), [-1, -c, -b, b, c, 1], atol=1e-15)


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5])
def test_basis_orthonormal_on_tetrahedron(N):
    pts, w = tet_quadrature(N + 2)
    assert abs(w.sum() - 4.0 / 3.0) < 1e-14          # volume of the reference tetrahedron
    Vq = R.vandermonde3d(N, pts)
    G = (Vq * w[:, None]).T @ Vq
    assert np.max(np.abs(G - np.eye(Vq.shape[1]))) < 1e-13


@pytest.mark.parametrize("N", [2, 4])
def test_basis_gradient_matches_difference_quotient(N):
    g = np.random.default_rng(0)
    lam = g.dirichlet(np.ones(4), size=20)
    pts = lam @ R.REF_VERTS
    h = 1e-6
    dr, ds, dt = R.grad_vandermonde3d(N, pts)
    for d, grad in enumerate((dr, ds, dt)):
        e = np.zeros(3)
        e[d] = h
        fd = (R.vandermonde3d(N, pts + e) - R.vandermonde3d(N, pts - e)) / (2 * h)
        assert np.max(np.abs(fd - grad)) < 1e-6 * max(1.0, np.max(np.abs(grad)))


@pytest.mark.parametrize("N", range(1, 10))
def test_D_is_exact_on_polynomials_of_degree_N(N):
    ref = R.ref_element(N)
    r, s, t = ref.rst.T
    worst = 0.0
    for p, q, m in itertools.product(range(N + 1), repeat=3):
        if p + q + m > N:
            continue
        f = r ** p * s ** q * t ** m
        fr = p * r ** max(p - 1, 0) * s ** q * t ** m
        fs = q * r ** p * s ** max(q - 1, 0) * t ** m
        ft = m * r ** p * s ** q * t ** max(m - 1, 0)
        for D, exact in ((ref.Dr, fr), (ref.Ds, fs), (ref.Dt, ft)):
            worst = max(worst, np.max(np.abs(D @ f - exact)))
    assert worst < 1e-12
    assert np.max(np.abs(ref.Dr @ np.ones(ref.Np))) < 1e-12


@pytest.mark.parametrize("N", range(1, 8))
def test_Ds_is_Dr_under_the_node_permutation_r_to_s(N):
    # Sec. 5.4 notes that the three differentiation matrices are similar under a permutation.
    ref = R.ref_element(N)
    swapped = ref.rst[:, [1, 0, 2]]
    d = np.linalg.norm(ref.rst[:, None, :] - swapped[None, :, :], axis=2)
    P = np.argmin(d, axis=1)
    assert np.max(np.min(d, axis=1)) < 1e-13
    assert np.max(np.abs(ref.Ds - ref.Dr[np.ix_(P, P)])) < 2e-12


# Fingerprints computed independently from the same node recipe while the design was
# surveyed (Frobenius norms, max entry, and sum of r^2 over the nodes).
FINGERPRINTS = {
    1: (1.4142135624, 0.5, 12.727922, 4.0),
    2: (7.0000000000, 2.0, 33.582920, 7.0),
    3: (18.8497503013, 4.0450849719, 67.086222, 12.533333333333),
    4: (39.7681740332, 6.7565024887, 115.253041, 20.678825572349),
    5: (73.1647369030, 10.1414159363, 182.436715, None),
    6: (123.9706051552, 14.2015766029, 271.651577, None),
    7: (203.7879530722, 18.9375986071, 388.316121, 65.484161300591),
}


@pytest.mark.parametrize("N", range(1, 8))
def test_operator_fingerprints(N):
    ref = R.ref_element(N)
    fro, mx, lift, r2 = FINGERPRINTS[N]
    for D in (ref.Dr, ref.Ds, ref.Dt):
        assert abs(np.linalg.norm(D) - fro) < 1e-9 * fro
    assert abs(np.max(np.abs(ref.Dr)) - mx) < 1e-9 * mx
    assert abs(np.linalg.norm(ref.LIFT) - lift) < 1e-6 * lift
    if r2 is not None:
        assert abs(np.sum(ref.rst[:, 0] ** 2) - r2) < 1e-11


@pytest.mark.parametrize("N", range(1, 8))
def test_node_set_properties(N):
    ref = R.ref_element(N)
    rst = ref.rst
    # exactly Nfp nodes on each face plane
    planes = [rst[:, 2] + 1, rst[:, 1] + 1, rst.sum(axis=1) + 1, rst[:, 0] + 1]
    for f, g in enumerate(planes):
        on = np.nonzero(np.abs(g) < 1e-12)[0]
        assert on.size == ref.Nfp
        assert np.array_equal(on, ref.Fmask[f])
    # nodes on the edge v1-v2 (s = t = -1) are the GLL points
    edge = np.nonzero((np.abs(rst[:, 1] + 1) < 1e-12) & (np.abs(rst[:, 2] + 1) < 1e-12))[0]
    assert np.max(np.abs(np.sort(rst[edge, 0]) - R.gll_points(N))) < 1e-14
    # invariance under r<->s and under the cyclic vertex permutation v2->v3->v4->v2
    bary = np.stack([-(1 + rst.sum(axis=1)) / 2, (1 + rst[:, 0]) / 2, (1 + rst[:, 1]) / 2,
                     (1 + rst[:, 2]) / 2], axis=1)
    for perm in ([0, 2, 1, 3], [0, 3, 1, 2], [1, 0, 2, 3]):
        pb = bary[:, perm]
        prst = np.stack([2 * pb[:, 1] - 1, 2 * pb[:, 2] - 1, 2 * pb[:, 3] - 1], axis=1)
        d = np.linalg.norm(rst[:, None, :] - prst[None, :, :], axis=2)
        assert np.max(np.min(d, axis=1)) < 5e-15


@pytest.mark.parametrize("N", [3, 5, 7])
def test_lebesgue_constant_beats_equispaced(N):
    ref = R.ref_element(N)
    g = np.random.default_rng(1)
    pts = g.dirichlet(np.ones(4), size=20000) @ R.REF_VERTS
    leb = np.max(np.sum(np.abs(lagrange_at(ref, pts)), axis=1))
    ijk = R.lattice(N)
    eq = -1 + 2 * ijk / N
    Veq = R.vandermonde3d(N, eq)
    leb_eq = np.max(np.sum(np.abs(R.vandermonde3d(N, pts) @ np.linalg.inv(Veq)), axis=1))
    assert leb < leb_eq
    if N >= 5:
        assert leb < 0.7 * leb_eq


@pytest.mark.parametrize("N", range(1, 7))
def test_mass_matrix_is_integral_of_lagrange_products(N):
    ref = R.ref_element(N)
    pts, w = tet_quadrature(N + 2)
    L = lagrange_at(ref, pts)
    Mq = (L * w[:, None]).T @ L
    assert np.max(np.abs(Mq - ref.M)) < 1e-13 * np.max(np.abs(ref.M)) * 10


@pytest.mark.parametrize("N", range(1, 7))
def test_lift_is_inverse_mass_times_face_integrals(N):
    """LIFT = M^-1 E with E[i,(f,j)] = integral over face f of l_i l_{Fmask_f[j]}, in the face's
    in-face reference coordinates (the area factor of the slanted face lives in sJ)."""
    ref = R.ref_element(N)
    pts2, w2 = tri_quadrature(N + 2)
    a, b = pts2[:, 0], pts2[:, 1]
    m1 = -np.ones_like(a)
    face_pts = [np.stack([a, b, m1], 1), np.stack([a, m1, b], 1),
                np.stack([-1 - a - b, a, b], 1), np.stack([m1, a, b], 1)]
    E = np.zeros((ref.Np, 4 * ref.Nfp))
    for f in range(4):
        L = lagrange_at(ref, face_pts[f])
        E[:, f * ref.Nfp:(f + 1) * ref.Nfp] = (L * w2[:, None]).T @ L[:, ref.Fmask[f]]
    lift = np.linalg.solve(ref.M, E)
    assert np.max(np.abs(lift - ref.LIFT)) < 5e-13 * np.max(np.abs(ref.LIFT))


def test_eoc_routine_reproduces_paper_table():
    h = np.array([0.3, 0.255, 0.21675, 0.184237])
    for row in read_golden("convergence_table.txt"):
        err = np.array([float(v) for v in row[1:5]])
        slope = np.polyfit(np.log(h), np.log(err), 1)[0]
        assert abs(slope - float(row[5])) <= 0.01

"""Pins of the oracle's Maxwell operator and time stepper.

P8  energy: the upwind operator is dissipative, the central one with PEC walls is skew.
P9  two-tetrahedron brute force: the operator equals an independent weak-form assembly with
    a monomial Lagrange basis and physical-space quadrature (no D, LIFT, Fscale or maps).
P10 the cavity eigenmode converges at order about N+1.
P11 the LSRK4 coefficients satisfy the fourth-order conditions.
P12 energy does not grow over time steps.
P13 element-permutation invariance; P14 linearity.
"""
import itertools
import math

import numpy as np
import pytest

import dginputs
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

from test_oracle_refelem import tet_quadrature, tri_quadrature


def assemble(mesh, **kw):
    """Dense operator A with rhs(u) = A u, by applying rhs to unit vectors."""
    n = 6 * mesh.K * mesh.ref.Np
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        A[:, j] = W.rhs(mesh, e.reshape(6, mesh.K, mesh.ref.Np), **kw).ravel()
    return A


def mass_weight(mesh):
    blocks = [mesh.J[k] * mesh.ref.M for k in range(mesh.K)]
    from scipy.linalg import block_diag
    Mk = block_diag(*blocks)
    return block_diag(*([Mk] * 6))


@pytest.mark.parametrize("N,n", [(1, 1), (2, 1), (3, 1)])
def test_upwind_operator_is_dissipative_central_is_skew(N, n):
    v, e = dginputs.kuhn_cube(n, jitter=0.1)
    m = Mm.Mesh(v, e, R.ref_element(N))
    Mw = mass_weight(m)
    A = assemble(m)
    S = Mw @ A + A.T @ Mw
    scale = np.linalg.norm(Mw @ A)
    assert np.max(np.linalg.eigvalsh(S)) <= 1e-12 * scale
    assert np.min(np.linalg.eigvalsh(S)) < -1e-3 * scale     # genuinely dissipative
    Ac = assemble(m, alpha=0.0)
    assert np.linalg.norm(Mw @ Ac + Ac.T @ Mw) <= 1e-12 * np.linalg.norm(Mw @ Ac)


# ---------------------------------------------------------------------------------------
# P9: independent weak-form assembly on two tetrahedra

def _monomials(N):
    return [(p, q, r) for p in range(N + 1) for q in range(N + 1 - p) for r in range(N + 1 - p - q)]


class _MonoBasis:
    """Lagrange basis of P_N on one physical element from monomials in scaled coordinates."""

    def __init__(self, N, nodes_xyz):
        self.exps = _monomials(N)
        self.c = nodes_xyz.mean(axis=0)
        self.h = np.max(np.ptp(nodes_xyz, axis=0))
        V = self._mono(nodes_xyz)
        self.C = np.linalg.inv(V)              # l_i = sum_j C[j, i] m_j

    def _mono(self, x):
        xi = (x - self.c) / self.h
        return np.stack([xi[:, 0] ** p * xi[:, 1] ** q * xi[:, 2] ** r for p, q, r in self.exps], axis=1)

    def _dmono(self, x, d):
        xi = (x - self.c) / self.h
        cols = []
        for e in self.exps:
            if e[d] == 0:
                cols.append(np.zeros(x.shape[0]))
                continue
            ee = list(e)
            ee[d] -= 1
            cols.append(e[d] * xi[:, 0] ** ee[0] * xi[:, 1] ** ee[1] * xi[:, 2] ** ee[2] / self.h)
        return np.stack(cols, axis=1)

    def val(self, x):
        return self._mono(x) @ self.C

    def grad(self, x):
        return [self._dmono(x, d) @ self.C for d in range(3)]


def _flux_dot_n(nv, uE, uH):
    """n.F(u) following Maxwell's equations: E rows -n x H, H rows n x E (vectors (3, q))."""
    return np.concatenate([-np.cross(nv.T, uH.T).T, np.cross(nv.T, uE.T).T])


def _flux_vol_dot_grad(uE, uH, g):
    """F(u) . grad(l) for each of the 6 rows; g is (3, q)."""
    Ex, Ey, Ez = uE
    Hx, Hy, Hz = uH
    gx, gy, gz = g
    return np.stack([-Hz * gy + Hy * gz, Hz * gx - Hx * gz, -Hy * gx + Hx * gy,
                     Ez * gy - Ey * gz, -Ez * gx + Ex * gz, Ey * gx - Ex * gy])


def brute_force_operator(vxyz, etov, N, eps=None, mu=None, absorb=None):
    """Weak form M (eps dE/dt, mu dH/dt) = int F(u).grad l - int (n.F)* l on every element,
    assembled with physical-space quadrature and the upwind flux of Sec. 6 written out with
    the impedances Z = sqrt(mu/eps), Y = 1/Z of both sides (vacuum by default). Unmatched
    faces mirror the trace (wall), or take a zero exterior state where absorb[k][f] is set."""
    ref = R.ref_element(N)
    m = Mm.Mesh(vxyz, etov, ref, compute_maps=False)
    K, Np = m.K, ref.Np
    eps = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64)
    mu = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64)
    Zk = np.sqrt(mu / eps)
    absorb = np.zeros((K, 4), dtype=bool) if absorb is None else np.asarray(absorb, dtype=bool)
    bases = [_MonoBasis(N, m.x[:, k, :].T) for k in range(K)]
    qv, wv = tet_quadrature(N + 2)
    qf, wf = tri_quadrature(N + 2)
    n = 6 * K * Np
    A = np.zeros((n, n))

    def idx(f, k):
        return f * K * Np + k * Np + np.arange(Np)

    for k in range(K):
        vk = m.vxyz[m.etov[k]]
        B = bases[k]
        # volume quadrature on the physical element
        lam = np.stack([-(1 + qv.sum(1)) / 2, (1 + qv[:, 0]) / 2, (1 + qv[:, 1]) / 2, (1 + qv[:, 2]) / 2], 1)
        xq = lam @ vk
        wq = wv * m.J[k]
        L = B.val(xq)
        G = B.grad(xq)
        Mk = (L * wq[:, None]).T @ L
        Minv = np.linalg.inv(Mk)
        # contribution of every input dof (field g, node j of element kk) to d/dt of (f, k)
        for g in range(6):
            for j in range(Np):
                # volume: u = e_(g,j) on element k
                uE = np.zeros((3, xq.shape[0]))
                uH = np.zeros((3, xq.shape[0]))
                (uE if g < 3 else uH)[g % 3] = L[:, j]
                vol = np.stack([(_flux_vol_dot_grad(uE, uH, [G[0][:, i], G[1][:, i], G[2][:, i]]) * wq).sum(1)
                                for i in range(Np)], axis=1)      # 6 x Np
                A[np.concatenate([idx(f, k) for f in range(6)]), g * K * Np + k * Np + j] += (Minv @ vol.T).T.ravel()
        # faces
        for f, fv in enumerate(R.FACE_VERTS):
            P = vk[list(fv)]
            lamf = np.stack([-(qf[:, 0] + qf[:, 1]) / 2, (1 + qf[:, 0]) / 2, (1 + qf[:, 1]) / 2], 1)
            xf = lamf @ P
            area = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
            wfa = wf * area / 2.0
            nv = np.cross(P[1] - P[0], P[2] - P[0])
            nv = nv / np.linalg.norm(nv)
            opp = vk[[i for i in range(4) if i not in fv][0]]
            if np.dot(nv, P[0] - opp) < 0:
                nv = -nv
            nvq = np.repeat(nv[:, None], xf.shape[0], 1)
            Lm = B.val(xf)
            # neighbour element: the other element owning this vertex triple
            key = sorted(m.etov[k][list(fv)])
            nb = None
            for kk in range(K):
                if kk == k:
                    continue
                for ff in R.FACE_VERTS:
                    if sorted(m.etov[kk][list(ff)]) == key:
                        nb = kk
            Lp = bases[nb].val(xf) if nb is not None else None
            sources = [(k, Lm, -1)] + ([(nb, Lp, +1)] if nb is not None else [])
            Zm = Zk[k]
            Zp = Zk[nb] if nb is not None else Zk[k]
            for src, Ls, side in sources:
                for g in range(6):
                    for j in range(Np):
                        um = np.zeros((6, xf.shape[0]))
                        up = np.zeros((6, xf.shape[0]))
                        if side < 0:
                            um[g] = Ls[:, j]
                            if nb is None and not absorb[k][f]:   # wall mirror
                                up[:3] = -um[:3]
                                up[3:] = um[3:]
                        else:
                            up[g] = Ls[:, j]
                        dE, dH = up[:3] - um[:3], up[3:] - um[3:]
                        # [n.F - (n.F)*] from Sec. 6: {Z}^-1 / 2 = 1 / (Z- + Z+)
                        bE = np.cross(nvq.T, (Zp * dH - np.cross(nvq.T, dE.T).T).T).T / (Zm + Zp)
                        bH = np.cross(nvq.T, (-dE / Zp - np.cross(nvq.T, dH.T).T).T).T / (1 / Zm + 1 / Zp)
                        star = _flux_dot_n(nvq, um[:3], um[3:]) - np.concatenate([bE, bH])
                        face = (star[:, :, None] * Lm[None, :, :] * wfa[None, :, None]).sum(1)  # 6 x Np
                        col = g * K * Np + src * Np + j
                        A[np.concatenate([idx(ff_, k) for ff_ in range(6)]), col] -= (Minv @ face.T).T.ravel()
    for k in range(K):
        for f in range(6):
            A[idx(f, k)] /= eps[k] if f < 3 else mu[k]
    return A, m


@pytest.mark.parametrize("N", [1, 2, 3])
def test_two_tet_brute_force(N):
    vxyz = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.05, 0.9, 0.1], [0.1, 0.0, 1.1],
                     [0.9, 0.8, 0.95]])
    etov = np.array([[0, 1, 2, 3], [1, 2, 3, 4]])
    A_bf, m = brute_force_operator(vxyz, Mm.orient(vxyz, etov), N)
    mo = Mm.Mesh(vxyz, etov, R.ref_element(N))
    A = assemble(mo)
    assert np.linalg.norm(A - A_bf) <= 1e-12 * np.linalg.norm(A)


# ---------------------------------------------------------------------------------------

def _cavity_error(N, n, T):
    ref = R.ref_element(N)
    v, e = dginputs.kuhn_cube(n)
    m = Mm.Mesh(v, e, ref)
    x, y, z = m.x
    u = dginputs.cavity_tm110(x, y, z, 0.0)
    ns = int(math.ceil(T / W.stable_dt(m)))
    dt = T / ns
    res = None
    for _ in range(ns):
        u, res = W.lsrk4_step(m, u, dt, res)
    err, _ = W.l2_error(m, u, dginputs.cavity_tm110(x, y, z, T))
    return err


@pytest.mark.slow
@pytest.mark.parametrize("N,meshes", [(1, (2, 4, 8)), (2, (1, 2, 4)), (3, (1, 2, 4)), (4, (1, 2))])
def test_cavity_mode_converges_at_order_N_plus_one(N, meshes):
    errs = [_cavity_error(N, n, 0.5) for n in meshes]
    rate = math.log(errs[-2] / errs[-1]) / math.log(meshes[-1] / meshes[-2])
    assert rate >= N + 0.5 if N > 1 else rate >= 1.5


def test_lsrk4_fourth_order_conditions():
    # Butcher tableau of the 2N-storage scheme: stage i evaluates at u + sum_j A_ij dt k_j.
    a, b = W.RK4A, W.RK4B
    s = 5
    # res_i = a_i res_{i-1} + dt k_i, u_i = u_{i-1} + b_i res_i; express res_i = sum_j R_ij k_j
    Rm = np.zeros((s, s))
    for i in range(s):
        if i > 0:
            Rm[i] = a[i] * Rm[i - 1]
        Rm[i, i] += 1.0
    U = np.zeros((s + 1, s))                  # u_i = u_0 + sum_j U_ij dt k_j
    for i in range(s):
        U[i + 1] = U[i] + b[i] * Rm[i]
    A = U[:s]                                  # stage i uses u_{i}
    bw = U[s]
    c = A.sum(1)
    conds = [bw.sum() - 1, bw @ c - 1 / 2, bw @ c ** 2 - 1 / 3, bw @ A @ c - 1 / 6,
             bw @ c ** 3 - 1 / 4, bw @ (c * (A @ c)) - 1 / 8, bw @ A @ c ** 2 - 1 / 12,
             bw @ A @ A @ c - 1 / 24]
    assert max(abs(x) for x in conds) < 1e-14
    assert np.max(np.abs(c - W.RK4C)) < 1e-15
    # stability polynomial coefficient of z^5
    assert abs(bw @ A @ A @ A @ c - 1 / 200) < 1e-4


@pytest.fixture(scope="module")
def small_jittered():
    v, e = dginputs.kuhn_cube(2, jitter=0.15, permute=True)
    return v, e, Mm.Mesh(v, e, R.ref_element(3))


def _smooth(m):
    x, y, z = m.x
    return dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x, y, z)


def test_energy_never_grows(small_jittered):
    _, _, m = small_jittered
    u = _smooth(m)
    dt = W.stable_dt(m)
    res = None
    e_prev = W.energy(m, u)
    for _ in range(50):
        u, res = W.lsrk4_step(m, u, dt, res)
        e_now = W.energy(m, u)
        assert e_now <= e_prev * (1 + 1e-14)
        e_prev = e_now


@pytest.mark.slow
def test_energy_never_grows_over_ten_thousand_steps():
    """P12 over 10^4 steps of a jittered 2^3 cube (N = 2, CFL 0.5): the upwind energy decays
    monotonically, step after step."""
    v, e = dginputs.kuhn_cube(2, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(2))
    u = _smooth(m)
    dt = W.stable_dt(m)
    res = None
    e_prev = e0 = W.energy(m, u)
    for _ in range(10000):
        u, res = W.lsrk4_step(m, u, dt, res)
        e_now = W.energy(m, u)
        assert e_now <= e_prev * (1 + 1e-14)
        e_prev = e_now
    assert 0.0 < e_prev < e0


def test_element_permutation_invariance(small_jittered):
    v, e, m = small_jittered
    g = np.random.default_rng(7)
    perm = g.permutation(m.K)
    mp = Mm.Mesh(v, e[perm], m.ref)
    u = _smooth(m)
    r = W.rhs(m, u)
    rp = W.rhs(mp, u[:, perm, :])
    assert np.array_equal(rp, r[:, perm, :])


def test_linearity(small_jittered):
    _, _, m = small_jittered
    g = np.random.default_rng(3)
    u = g.standard_normal((6, m.K, m.ref.Np))
    w = g.standard_normal((6, m.K, m.ref.Np))
    lhs = W.rhs(m, 2.5 * u - 0.75 * w)
    rhs = 2.5 * W.rhs(m, u) - 0.75 * W.rhs(m, w)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14 * np.max(np.abs(lhs)) * 10


def test_rhs_of_cavity_mode_is_its_time_derivative():
    errs = []
    for n in (2, 4):
        v, e = dginputs.kuhn_cube(n)
        m = Mm.Mesh(v, e, R.ref_element(3))
        x, y, z = m.x
        w = math.pi * math.sqrt(2.0)
        u0 = dginputs.cavity_tm110(x, y, z, 0.0)
        # d/dt at t = 0: E' = 0, H' = w * (H at t = pi/(2w))
        dudt = w * dginputs.cavity_tm110(x, y, z, math.pi / (2 * w))
        dudt[:3] = 0.0
        err, nrm = W.l2_error(m, W.rhs(m, u0), dudt)
        errs.append(err / nrm)
    assert errs[1] < errs[0] / 6.0


def test_sampled_rhs_and_step_equal_the_full_ones(small_jittered):
    _, _, m = small_jittered
    u = _smooth(m)
    idx = np.array([0, 5, 17, 40])
    assert np.array_equal(W.rhs_at(m, u, idx), W.rhs(m, u)[:, idx])
    dt = W.stable_dt(m)
    full, _ = W.lsrk4_step(m, u, dt)
    assert np.array_equal(W.lsrk4_step_at(m, u, dt, idx), full[:, idx])


def test_rhs_on_element_ranges_equals_the_full_one(small_jittered):
    _, _, m = small_jittered
    u = _smooth(m)
    parts = [W.rhs_range(m, u, a, b) for a, b in ((0, 5), (5, 6), (6, 31), (31, m.K))]
    assert np.array_equal(np.concatenate(parts, axis=1), W.rhs(m, u))

"""Oracle Maxwell right-hand side, LSRK4 step and energy (test infrastructure only).

Semi-discrete operator (Sec. 2, eq. semidiscrete-dg):
    du/dt = - sum_nu D^nu F(u) + L [ n.F - (n.F)* ]
for Maxwell's equations in vacuum or a linear isotropic medium (Sec. 6, eq. maxwells-claws):
    eps dE/dt = curl H,   mu dH/dt = - curl E.
The volume term is therefore (curl H / eps, -curl E / mu). The paper's printed flux matrix
F(u) has the E and H column blocks exchanged relative to these equations; this oracle follows
the equations (and the printed upwind flux, which is consistent with them).

Surface term, upwind flux of Sec. 6 with jump [u] = u+ - u- (penalty alpha = 1 is the upwind
flux; alpha = 0 is the central flux, used only by the energy tests):
    [n.F - (n.F)*]_E = 1/(Z- + Z+) n x ( Z+ [H] - alpha n x [E] )
    [n.F - (n.F)*]_H = 1/(Y- + Y+) n x ( -Y+ [E] - alpha n x [H] )
which in vacuum is  1/2 (n x [H] + alpha([E] - (n.[E]) n))  and
                    1/2 (-n x [E] + alpha([H] - (n.[H]) n)).
A perfectly conducting wall (Sec. 6 cavity) mirrors the trace: E+ = -E-, H+ = H-.

Time stepping: the five-stage fourth-order 2N-storage Runge-Kutta method of Carpenter and
Kennedy cited in Sec. 6: res <- a_i res + dt L(u); u <- u + b_i res.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh

# Carpenter-Kennedy (1994) five-stage, fourth-order, 2N-storage coefficients.
RK4A = np.array([0.0,
                 -567301805773.0 / 1357537059087.0,
                 -2404267990393.0 / 2016746695238.0,
                 -3550918686646.0 / 2091501179385.0,
                 -1275806237668.0 / 842570457699.0])
RK4B = np.array([1432997174477.0 / 9575080441755.0,
                 5161836677717.0 / 13612068292357.0,
                 1720146321549.0 / 2090206949498.0,
                 3134564353537.0 / 4481467310338.0,
                 2277821191437.0 / 14882151754819.0])
RK4C = np.array([0.0,
                 1432997174477.0 / 9575080441755.0,
                 2526269341429.0 / 6820363962896.0,
                 2006345519317.0 / 3224310063776.0,
                 2802321613138.0 / 2924317926251.0])


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def volume_term(mesh: Mesh, u):
    """(curl H, -curl E) at the nodes; u is (6, K, Np). Physical derivatives are
    d/dx_nu = sum_mu (d r_mu/d x_nu) D_mu, constant per element."""
    ref = mesh.ref
    D = (ref.Dr, ref.Ds, ref.Dt)
    # reference derivatives: (3 dirs, 6 fields, K, Np)
    ref_d = np.stack([np.einsum("ij,fkj->fki", Dm, u) for Dm in D])
    # physical derivatives: (3 dims nu, 6 fields, K, Np)
    phys = np.einsum("kmn,mfki->nfki", mesh.G, ref_d)
    dx, dy, dz = phys[0], phys[1], phys[2]
    Ex, Ey, Ez, Hx, Hy, Hz = range(6)
    curlH = np.stack([dy[Hz] - dz[Hy], dz[Hx] - dx[Hz], dx[Hy] - dy[Hx]])
    curlE = np.stack([dy[Ez] - dz[Ey], dz[Ex] - dx[Ez], dx[Ey] - dy[Ex]])
    return np.concatenate([curlH, -curlE])


def surface_flux(mesh: Mesh, u, alpha=1.0, eps=None, mu=None):
    """[n.F - (n.F)*] at every face node, (6, K, 4, Nfp), not yet scaled by Fscale."""
    K, Np = u.shape[1], u.shape[2]
    flat = u.reshape(6, K * Np)
    uM = flat[:, mesh.vmapM]
    uP = flat[:, mesh.vmapP]
    bnd = mesh.boundary[:, :, None]
    # perfectly conducting wall: E+ = -E-, H+ = H-
    uP = np.where(bnd[None], np.concatenate([-uM[:3], uM[3:]]), uP)
    dE = uP[:3] - uM[:3]
    dH = uP[3:] - uM[3:]
    n = np.moveaxis(mesh.n, 2, 0)[:, :, :, None]  # 3, K, 4, 1
    if eps is None and mu is None:
        zm = zp = ym = yp = np.ones((K, 4, 1))
    else:
        eps = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64)
        mu = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64)
        Z = np.sqrt(mu / eps)
        nbr = mesh.EToE
        zm = np.broadcast_to(Z[:, None, None], (K, 4, 1))
        zp = Z[nbr][:, :, None]
        ym, yp = 1.0 / zm, 1.0 / zp
    fE = _cross(n, zp * dH - alpha * _cross(n, dE)) / (zm + zp)
    fH = _cross(n, -yp * dE - alpha * _cross(n, dH)) / (ym + yp)
    return np.concatenate([fE, fH])


def rhs(mesh: Mesh, u, alpha=1.0, eps=None, mu=None):
    """Semi-discrete right-hand side du/dt, u of shape (6, K, Np), FP64."""
    ref = mesh.ref
    K, Np, Nfp = u.shape[1], ref.Np, ref.Nfp
    vol = volume_term(mesh, u)
    flux = surface_flux(mesh, u, alpha, eps, mu)                    # 6, K, 4, Nfp
    scaled = (flux * mesh.Fscale[None, :, :, None]).reshape(6, K, 4 * Nfp)
    lift = np.einsum("ij,fkj->fki", ref.LIFT, scaled)
    out = vol + lift
    if eps is not None or mu is not None:
        e = np.ones(K) if eps is None else np.asarray(eps, dtype=np.float64)
        m = np.ones(K) if mu is None else np.asarray(mu, dtype=np.float64)
        out[:3] /= e[None, :, None]
        out[3:] /= m[None, :, None]
    return out


def lsrk4_step(mesh: Mesh, u, dt, res=None, **kw):
    """One five-stage low-storage RK4 step; returns (u_new, res_new)."""
    u = np.array(u, dtype=np.float64, copy=True)
    res = np.zeros_like(u) if res is None else np.array(res, dtype=np.float64, copy=True)
    for a, b in zip(RK4A, RK4B):
        res = a * res + dt * rhs(mesh, u, **kw)
        u = u + b * res
    return u, res


def energy(mesh: Mesh, u, eps=None, mu=None):
    """1/2 sum_k J_k sum_fields u_k^T M u_k (eps, mu weights for E and H)."""
    M = mesh.ref.M
    per = np.einsum("fki,ij,fkj->fk", u, M, u)
    w = np.ones((6, mesh.K))
    if eps is not None:
        w[:3] *= np.asarray(eps)[None, :]
    if mu is not None:
        w[3:] *= np.asarray(mu)[None, :]
    return 0.5 * float(np.sum(w * per * mesh.J[None, :]))


def stable_dt(mesh: Mesh, cfl=0.5):
    """dt = cfl * min over faces of 1/Fscale, divided by N^2."""
    return cfl * float(np.min(1.0 / mesh.Fscale)) / mesh.ref.N ** 2


def l2_error(mesh: Mesh, u, uref):
    """Mass-weighted L2 norms over all six fields: (||u - uref||, ||uref||)."""
    def nrm(v):
        return float(np.sqrt(np.einsum("fki,ij,fkj,k->", v, mesh.ref.M, v, mesh.J)))
    return nrm(u - uref), nrm(uref)

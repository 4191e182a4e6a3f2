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
An absorbing face (the characteristic absorbing condition named for the scattering example of
Sec. 6) takes a zero exterior state, u+ = 0, with the exterior impedance equal to the interior
one; the upwind flux then lets outgoing characteristics leave and admits nothing.

Scattered-field form (the incident-field formulation of the scattering example of Sec. 6):
the unknown is the scattered field u_s = u - u_inc, where u_inc is a known incident plane
wave that solves Maxwell's equations in vacuum. The volume operator and interior fluxes are
unchanged (the operator is linear and u_inc is continuous); on a scatterer face the total field
meets the perfectly conducting wall, E_s+ + E_inc = -(E_s- + E_inc) and H_s+ = H_s-, so the
jump there is [E] = -2 (E_s- + E_inc(x, t)), [H] = 0. The operator then depends on t, and the
Runge-Kutta stages evaluate it at t + c_i dt.

Time stepping: the five-stage fourth-order 2N-storage Runge-Kutta method of Carpenter and
Kennedy cited in Sec. 6: res <- a_i res + dt L(u, t + c_i dt); u <- u + b_i res.
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


class PlaneWave:
    """Incident plane wave in vacuum: E = p f(k.x - t), H = (k x p) f(k.x - t), with unit
    direction k, polarisation p orthogonal to k and profile
    f(s) = c0 + c1 s + c2 sin(c3 s + c4). Any such field solves Maxwell's equations in vacuum
    (unit wave speed and impedance)."""

    def __init__(self, k, p, c):
        self.k = np.asarray(k, dtype=np.float64)
        self.p = np.asarray(p, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        assert self.k.shape == (3,) and self.p.shape == (3,) and self.c.shape == (5,)
        assert abs(np.linalg.norm(self.k) - 1.0) < 1e-12 and abs(self.k @ self.p) < 1e-12

    def profile(self, s):
        c0, c1, c2, c3, c4 = self.c
        return c0 + c1 * s + c2 * np.sin(c3 * s + c4)

    def fields(self, x, y, z, t):
        """(6, ...) incident field at the points (x, y, z) and time t."""
        f = self.profile(self.k[0] * x + self.k[1] * y + self.k[2] * z - t)
        h = np.cross(self.k, self.p)
        return np.stack([self.p[0] * f, self.p[1] * f, self.p[2] * f, h[0] * f, h[1] * f, h[2] * f])


def _cross(a, b):
    return np.stack([a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _curl_term(ref, G, u):
    """(curl H, -curl E) at the nodes of u (6, k, Np) with inverse-map derivatives G (k,3,3).
    Physical derivatives are d/dx_nu = sum_mu (d r_mu/d x_nu) D_mu, constant per element."""
    D = (ref.Dr, ref.Ds, ref.Dt)
    # reference derivatives: (3 dirs, 6 fields, k, Np)
    ref_d = np.stack([np.einsum("ij,fkj->fki", Dm, u) for Dm in D])
    # physical derivatives: (3 dims nu, 6 fields, k, Np)
    phys = np.einsum("kmn,mfki->nfki", G, ref_d)
    dx, dy, dz = phys[0], phys[1], phys[2]
    Ex, Ey, Ez, Hx, Hy, Hz = range(6)
    curlH = np.stack([dy[Hz] - dz[Hy], dz[Hx] - dx[Hz], dx[Hy] - dy[Hx]])
    curlE = np.stack([dy[Ez] - dz[Ey], dz[Ex] - dx[Ez], dx[Ey] - dy[Ex]])
    return np.concatenate([curlH, -curlE])


def volume_term(mesh: Mesh, u):
    """(curl H, -curl E) at the nodes; u is (6, K, Np)."""
    return _curl_term(mesh.ref, mesh.G, u)


def _flux_terms(flat, vM, vP, bnd, nrm, alpha, imp, absorb=None, scatter=None, einc=None):
    """[n.F - (n.F)*] at face nodes given flat fields (6, K*Np), maps vM/vP (k,4,Nfp),
    wall flags bnd (k,4), normals nrm (k,4,3), impedances imp = (zm, zp, ym, yp),
    absorbing-face flags absorb (k,4, a subset of the walls; None = none), scatterer-face
    flags scatter (k,4, walls) and the incident E at the face nodes einc (3,k,4,Nfp)."""
    uM = flat[:, vM]
    uP = flat[:, vP]
    b = bnd[:, :, None]
    # perfectly conducting wall: E+ = -E-, H+ = H-
    uP = np.where(b[None], np.concatenate([-uM[:3], uM[3:]]), uP)
    if absorb is not None:
        # absorbing face: zero exterior state
        uP = np.where(np.asarray(absorb, dtype=bool)[None, :, :, None], 0.0, uP)
    if scatter is not None:
        # scatterer face: the total field meets the wall, E+ = -E- - 2 E_inc, H+ = H-
        sc = np.asarray(scatter, dtype=bool)[None, :, :, None]
        uP = np.where(sc, np.concatenate([-uM[:3] - 2.0 * einc, uM[3:]]), uP)
    dE = uP[:3] - uM[:3]
    dH = uP[3:] - uM[3:]
    n = np.moveaxis(nrm, 2, 0)[:, :, :, None]  # 3, k, 4, 1
    zm, zp, ym, yp = imp
    fE = _cross(n, zp * dH - alpha * _cross(n, dE)) / (zm + zp)
    fH = _cross(n, -yp * dE - alpha * _cross(n, dH)) / (ym + yp)
    return np.concatenate([fE, fH])


def _impedances(mesh, elems, eps, mu):
    k = elems.size
    if eps is None and mu is None:
        one = np.ones((k, 4, 1))
        return one, one, one, one
    eps = np.ones(mesh.K) if eps is None else np.asarray(eps, dtype=np.float64)
    mu = np.ones(mesh.K) if mu is None else np.asarray(mu, dtype=np.float64)
    Z = np.sqrt(mu / eps)
    zm = np.broadcast_to(Z[elems][:, None, None], (k, 4, 1))
    zp = Z[mesh.EToE[elems]][:, :, None]
    return zm, zp, 1.0 / zm, 1.0 / zp


def _check_absorb(mesh: Mesh, absorb):
    if absorb is None:
        return None
    absorb = np.asarray(absorb, dtype=bool)
    assert absorb.shape == (mesh.K, 4) and not np.any(absorb & ~mesh.boundary), \
        "absorbing flags must mark boundary faces"
    return absorb


def _incident_at_faces(mesh: Mesh, vM, scatter, incident, t):
    """Incident E at the face nodes vM (3, k, 4, Nfp) at time t, or None without scatterers."""
    if scatter is None:
        return None
    x = mesh.x.reshape(3, -1)[:, vM]
    if incident is None:
        return np.zeros_like(x)
    return incident.fields(x[0], x[1], x[2], t)[:3]


def surface_flux(mesh: Mesh, u, alpha=1.0, eps=None, mu=None, absorb=None, scatter=None,
                 incident=None, t=0.0):
    """[n.F - (n.F)*] at every face node, (6, K, 4, Nfp), not yet scaled by Fscale."""
    K, Np = u.shape[1], u.shape[2]
    elems = np.arange(K)
    scatter = _check_absorb(mesh, scatter)
    return _flux_terms(u.reshape(6, K * Np), mesh.vmapM, mesh.vmapP, mesh.boundary, mesh.n, alpha,
                       _impedances(mesh, elems, eps, mu), _check_absorb(mesh, absorb), scatter,
                       _incident_at_faces(mesh, mesh.vmapM, scatter, incident, t))


def _assemble(ref, vol, flux, Fscale, eps_k, mu_k):
    k, Nfp = vol.shape[1], ref.Nfp
    scaled = (flux * Fscale[None, :, :, None]).reshape(6, k, 4 * Nfp)
    out = vol + np.einsum("ij,fkj->fki", ref.LIFT, scaled)
    if eps_k is not None:
        out[:3] /= eps_k[None, :, None]
    if mu_k is not None:
        out[3:] /= mu_k[None, :, None]
    return out


def rhs(mesh: Mesh, u, alpha=1.0, eps=None, mu=None, absorb=None, scatter=None, incident=None, t=0.0):
    """Semi-discrete right-hand side du/dt, u of shape (6, K, Np), FP64. eps, mu: per-element
    permittivity and permeability (None = 1); absorb: (K, 4) absorbing-face flags; scatter:
    (K, 4) scatterer-face flags of the scattered-field form, with the incident PlaneWave
    `incident` (None = no incident field) at time t."""
    vol = volume_term(mesh, u)
    flux = surface_flux(mesh, u, alpha, eps, mu, absorb, scatter, incident, t)   # 6, K, 4, Nfp
    e = None if eps is None else np.asarray(eps, dtype=np.float64)
    m = None if mu is None else np.asarray(mu, dtype=np.float64)
    return _assemble(mesh.ref, vol, flux, mesh.Fscale, e, m)


def rhs_at(mesh: Mesh, u, elems, alpha=1.0, eps=None, mu=None, absorb=None, scatter=None,
           incident=None, t=0.0):
    """The same right-hand side evaluated only at the elements `elems`: (6, len, Np). Face
    maps are computed for those elements only, so the mesh may be built with
    compute_maps=False. eps, mu (per element, None = 1), absorb ((K, 4) absorbing-face
    flags), scatter, incident and t as in rhs()."""
    from .mesh import face_maps
    elems = np.asarray(elems, dtype=np.int64)
    ref = mesh.ref
    K, Np = u.shape[1], u.shape[2]
    vol = _curl_term(ref, mesh.G[elems], u[:, elems, :])
    vM, vP = face_maps(mesh.x, mesh.EToE, mesh.EToF, ref.Fmask, elems)
    absorb = _check_absorb(mesh, absorb)
    scatter = _check_absorb(mesh, scatter)
    sc = None if scatter is None else scatter[elems]
    flux = _flux_terms(u.reshape(6, K * Np), vM, vP, mesh.boundary[elems], mesh.n[elems], alpha,
                       _impedances(mesh, elems, eps, mu), None if absorb is None else absorb[elems],
                       sc, _incident_at_faces(mesh, vM, sc, incident, t))
    e = None if eps is None else np.asarray(eps, dtype=np.float64)[elems]
    m = None if mu is None else np.asarray(mu, dtype=np.float64)[elems]
    return _assemble(ref, vol, flux, mesh.Fscale[elems], e, m)


def rhs_range(mesh: Mesh, u, k0, k1, alpha=1.0):
    """The right-hand side (vacuum) at elements k0 .. k1-1 of a mesh built with its face maps,
    (6, k1 - k0, Np): the same arithmetic as rhs() on a contiguous range of elements, so that
    disjoint ranges can be evaluated on separate host cores."""
    sl = slice(k0, k1)
    ref = mesh.ref
    K, Np = u.shape[1], u.shape[2]
    vol = _curl_term(ref, mesh.G[sl], u[:, sl, :])
    flux = _flux_terms(u.reshape(6, K * Np), mesh.vmapM[sl], mesh.vmapP[sl], mesh.boundary[sl], mesh.n[sl],
                       alpha, _impedances(mesh, np.arange(k0, k1), None, None))
    return _assemble(ref, vol, flux, mesh.Fscale[sl], None, None)


def lsrk4_step(mesh: Mesh, u, dt, res=None, t=0.0, **kw):
    """One five-stage low-storage RK4 step from time t; returns (u_new, res_new). Stage i
    evaluates the right-hand side at t + c_i dt (only the scattered-field form depends on t)."""
    u = np.array(u, dtype=np.float64, copy=True)
    res = np.zeros_like(u) if res is None else np.array(res, dtype=np.float64, copy=True)
    for a, b, c in zip(RK4A, RK4B, RK4C):
        res = a * res + dt * rhs(mesh, u, t=t + c * dt, **kw)
        u = u + b * res
    return u, res


def face_rings(mesh: Mesh, elems, depth):
    """Sets S_0 = elems, S_d = S_{d-1} plus its face neighbours, for d = 0..depth."""
    rings = [np.unique(np.asarray(elems, dtype=np.int64))]
    for _ in range(depth):
        prev = rings[-1]
        rings.append(np.unique(np.concatenate([prev, mesh.EToE[prev].ravel()])))
    return rings


def lsrk4_step_at(mesh: Mesh, u, dt, elems, alpha=1.0, t=0.0, **kw):
    """One LSRK4 step from res = 0, evaluated only where it is needed for `elems`.

    A stage's right-hand side at an element reads only that element and its face neighbours,
    so after five stages the result at `elems` depends on the elements within five face
    steps. Stage i (1..5) evaluates the right-hand side and updates res and u on the ring of
    depth 5 - i; everything read there was updated at the previous stage. Returns u at
    `elems` (6, len, Np), identical to lsrk4_step(...)[0][:, elems]."""
    rings = face_rings(mesh, elems, 5)
    u = np.array(u, dtype=np.float64, copy=True)
    res = np.zeros_like(u)
    for i, (a, b, c) in enumerate(zip(RK4A, RK4B, RK4C)):
        S = rings[4 - i]
        r = rhs_at(mesh, u, S, alpha, t=t + c * dt, **kw)
        res[:, S] = a * res[:, S] + dt * r
        u[:, S] = u[:, S] + b * res[:, S]
    return u[:, np.asarray(elems, dtype=np.int64)]


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
        return float(np.sqrt(np.einsum("fki,ij,fkj,k->", v, mesh.ref.M, v, mesh.J, optimize=True)))
    return nrm(u - uref), nrm(uref)

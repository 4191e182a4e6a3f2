"""Oracle reference tetrahedron (test infrastructure only; never part of the product path).

Sec. 2 of the paper expands the solution in the Lagrange basis of P_N on interpolation nodes
(the warp-and-blend nodes it cites) and defines the mass, stiffness, differentiation and face
mass matrices (eq. dg-global-matrices) and the lifting matrix L = M^-1 [M^A1 .. M^A4]
(Fig. lifting-matrix). On affine simplices these are reference matrices (eq.
dg-reference-matrices); this module builds them on the reference tetrahedron in FP64.

Conventions the paper leaves open (they change layout, not values):
  vertices v1=(-1,-1,-1), v2=(1,-1,-1), v3=(-1,1,-1), v4=(-1,-1,1);
  faces F1=(v1,v2,v3) t=-1, F2=(v1,v2,v4) s=-1, F3=(v2,v3,v4) r+s+t=-1, F4=(v1,v3,v4) r=-1;
  node lattice (i,j,k), i+j+k<=N, ordered k outermost, then j, then i innermost;
  Fmask lists the nodes of each face in ascending node index.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np

# Warp-and-blend blending exponents alpha_opt(N), N = 1..15 (Warburton 2006, tetrahedron).
ALPHA_OPT = [0.0, 0.0, 0.0, 0.1002, 1.1332, 1.5608, 1.3413, 1.2577, 1.1603, 1.10153,
             0.6080, 0.4523, 0.8856, 0.8717, 0.9655]

REF_VERTS = np.array([[-1.0, -1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, 1.0, -1.0],
                      [-1.0, -1.0, 1.0]])
# local vertex triples of the faces (0-based) and the vertex opposite each face
FACE_VERTS = [(0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3)]
FACE_OPPOSITE = [3, 2, 0, 1]

NODE_TOL = 1e-10


def counts(N: int):
    """(Np, Nfp) for order N: dim P_N in 3D and 2D."""
    return (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2


# ----------------------------------------------------------------------------------------
# one-dimensional building blocks

def jacobi_normalized(x, alpha: float, beta: float, n: int):
    """Orthonormal Jacobi polynomial of degree n for weight (1-x)^alpha (1+x)^beta on [-1,1].

    Three-term recurrence of the orthonormal family: x p_m = a_{m+1} p_{m+1} + b_m p_m
    + a_m p_{m-1}, with p_0 = 1/sqrt(integral of the weight).
    """
    x = np.asarray(x, dtype=np.float64)
    ab = alpha + beta
    w0 = 2.0 ** (ab + 1.0) * math.gamma(alpha + 1.0) * math.gamma(beta + 1.0) / math.gamma(ab + 2.0)
    p_prev = np.zeros_like(x)
    p = np.full_like(x, 1.0 / math.sqrt(w0))
    if n == 0:
        return p

    def a_coef(m):  # off-diagonal entry a_m, m >= 1
        s = 2.0 * m + ab
        return 2.0 / s * math.sqrt(m * (m + ab) * (m + alpha) * (m + beta) / ((s - 1.0) * (s + 1.0)))

    def b_coef(m):  # diagonal entry b_m
        if m == 0:
            return (beta - alpha) / (ab + 2.0)
        s = 2.0 * m + ab
        return (beta * beta - alpha * alpha) / (s * (s + 2.0))

    for m in range(n):
        a_next = a_coef(m + 1)
        a_cur = a_coef(m) if m > 0 else 0.0
        p_next = ((x - b_coef(m)) * p - a_cur * p_prev) / a_next
        p_prev, p = p, p_next
    return p


def jacobi_normalized_deriv(x, alpha: float, beta: float, n: int):
    """d/dx of the orthonormal Jacobi polynomial: sqrt(n(n+a+b+1)) p_{n-1}^{(a+1,b+1)}."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return math.sqrt(n * (n + alpha + beta + 1.0)) * jacobi_normalized(x, alpha + 1.0, beta + 1.0, n - 1)


def gauss_jacobi(alpha: float, beta: float, n: int):
    """n-point Gauss-Jacobi rule (points, weights) by the Golub-Welsch eigenvalue method."""
    ab = alpha + beta
    diag = np.empty(n)
    off = np.empty(max(n - 1, 0))
    for m in range(n):
        if m == 0:
            diag[m] = (beta - alpha) / (ab + 2.0)
        else:
            s = 2.0 * m + ab
            diag[m] = (beta * beta - alpha * alpha) / (s * (s + 2.0))
    for m in range(1, n):
        s = 2.0 * m + ab
        off[m - 1] = 2.0 / s * math.sqrt(m * (m + ab) * (m + alpha) * (m + beta) / ((s - 1.0) * (s + 1.0)))
    jm = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
    pts, vecs = np.linalg.eigh(jm)
    mu0 = 2.0 ** (ab + 1.0) * math.gamma(alpha + 1.0) * math.gamma(beta + 1.0) / math.gamma(ab + 2.0)
    wts = mu0 * vecs[0, :] ** 2
    return pts, wts


def gll_points(N: int):
    """N+1 Gauss-Lobatto-Legendre points on [-1,1]: the end points and the zeros of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    inner, _ = gauss_jacobi(1.0, 1.0, N - 1)
    return np.concatenate([[-1.0], np.sort(inner), [1.0]])


def warp_factor(N: int, x):
    """Edge warp divided by the edge bubble.

    w(x) = sum_i (x_i^GLL - x_i^eq) l_i^eq(x) moves equispaced points to GLL points; the
    returned value is w(x)/(1-x^2) in the interior and 0 at the end points (where w vanishes).
    """
    x = np.asarray(x, dtype=np.float64)
    xeq = np.linspace(-1.0, 1.0, N + 1)
    xg = gll_points(N)
    w = np.zeros_like(x)
    for i in range(N + 1):
        li = np.ones_like(x)
        for j in range(N + 1):
            if j != i:
                li = li * (x - xeq[j]) / (xeq[i] - xeq[j])
        w = w + (xg[i] - xeq[i]) * li
    inner = np.abs(x) < 1.0 - NODE_TOL
    out = np.zeros_like(x)
    out[inner] = w[inner] / (1.0 - x[inner] ** 2)
    return out


# ----------------------------------------------------------------------------------------
# nodes

def lattice(N: int):
    """Integer lattice (i, j, k), i+j+k <= N, k outermost, j, i innermost; shape (Np, 3)."""
    out = [(i, j, k) for k in range(N + 1) for j in range(N + 1 - k) for i in range(N + 1 - k - j)]
    return np.array(out, dtype=np.int64)


def _triangle_shift(N, alpha, lam, pts):
    """Warp of a face: sum over the three edges (p,q) opposite o of the face of
    4 lam_p lam_q warp_factor(lam_q - lam_p) (1 + (alpha lam_o)^2) (P_q - P_p)/|P_q - P_p|."""
    shift = np.zeros((lam[0].size, 3))
    for p, q, o in ((1, 2, 0), (2, 0, 1), (0, 1, 2)):
        d = pts[q] - pts[p]
        d = d / np.linalg.norm(d)
        mag = 4.0 * lam[p] * lam[q] * warp_factor(N, lam[q] - lam[p]) * (1.0 + (alpha * lam[o]) ** 2)
        shift += mag[:, None] * d[None, :]
    return shift


def nodes(N: int):
    """Warp-and-blend interpolation nodes (r, s, t) on the reference tetrahedron, (Np, 3).

    Built on an equilateral tetrahedron: every face warps its equispaced lattice toward the
    1D GLL distribution along each edge, blended into the volume; then mapped back to (r,s,t).
    """
    alpha = ALPHA_OPT[N - 1] if N <= 15 else 1.0
    ijk = lattice(N)
    bary = np.stack([1.0 - ijk.sum(axis=1) / N, ijk[:, 0] / N, ijk[:, 1] / N, ijk[:, 2] / N], axis=1)
    s3, s6 = math.sqrt(3.0), math.sqrt(6.0)
    veq = np.array([[-1.0, -1.0 / s3, -1.0 / s6], [1.0, -1.0 / s3, -1.0 / s6],
                    [0.0, 2.0 / s3, -1.0 / s6], [0.0, 0.0, 3.0 / s6]])
    xeq = bary @ veq
    shift = np.zeros_like(xeq)
    for f in range(4):
        a = FACE_OPPOSITE[f]
        b, c, d = FACE_VERTS[f]
        la = bary[:, a]
        lam = [bary[:, b], bary[:, c], bary[:, d]]
        tri = _triangle_shift(N, alpha, lam, [veq[b], veq[c], veq[d]])
        denom = (lam[0] + 0.5 * la) * (lam[1] + 0.5 * la) * (lam[2] + 0.5 * la)
        blend = np.zeros_like(la)
        ok = denom > NODE_TOL
        blend[ok] = (1.0 + (alpha * la[ok]) ** 2) * lam[0][ok] * lam[1][ok] * lam[2][ok] / denom[ok]
        shift += blend[:, None] * tri
        npos = (lam[0] > NODE_TOL).astype(int) + (lam[1] > NODE_TOL) + (lam[2] > NODE_TOL)
        edge = (la < NODE_TOL) & (npos < 3)
        shift[edge] = tri[edge]
    xw = xeq + shift
    # barycentrics of the warped points w.r.t. the equilateral vertices, then (r,s,t)
    amat = np.vstack([veq.T, np.ones(4)])
    rhs = np.vstack([xw.T, np.ones(xw.shape[0])])
    lw = np.linalg.solve(amat, rhs).T
    return np.stack([-1.0 + 2.0 * lw[:, 1], -1.0 + 2.0 * lw[:, 2], -1.0 + 2.0 * lw[:, 3]], axis=1)


def face_masks(N: int):
    """Node indices on each face F1..F4 in ascending order, by the integer lattice."""
    ijk = lattice(N)
    i, j, k = ijk[:, 0], ijk[:, 1], ijk[:, 2]
    on = [k == 0, j == 0, i + j + k == N, i == 0]
    return np.array([np.nonzero(m)[0] for m in on], dtype=np.int64)


# ----------------------------------------------------------------------------------------
# orthonormal basis (collapsed coordinates)

def _rst_to_abc(r, s, t, tol=1e-12):
    a = np.full_like(r, -1.0)
    st = -(s + t)
    ok = np.abs(st) > tol
    a[ok] = 2.0 * (1.0 + r[ok]) / st[ok] - 1.0
    b = np.full_like(r, -1.0)
    ok = np.abs(1.0 - t) > tol
    b[ok] = 2.0 * (1.0 + s[ok]) / (1.0 - t[ok]) - 1.0
    return a, b, t.copy()


def _pw(x, p):
    """x**p for integer p >= 0; returns zeros for p < 0 (only ever met with a zero factor)."""
    if p < 0:
        return np.zeros_like(x)
    return x ** p


def basis_modes(N: int):
    """Multi-indices (i, j, k), i+j+k <= N, of the orthonormal basis."""
    return [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i) for k in range(N + 1 - i - j)]


def basis3d(r, s, t, i, j, k):
    """psi_ijk = 2 sqrt2 P_i(a) P_j^(2i+1,0)(b) (1-b)^i P_k^(2i+2j+2,0)(c) (1-c)^(i+j)."""
    a, b, c = _rst_to_abc(r, s, t)
    return (2.0 * math.sqrt(2.0) * jacobi_normalized(a, 0, 0, i)
            * jacobi_normalized(b, 2 * i + 1, 0, j) * _pw(1.0 - b, i)
            * jacobi_normalized(c, 2 * i + 2 * j + 2, 0, k) * _pw(1.0 - c, i + j))


def grad_basis3d(r, s, t, i, j, k):
    """(d/dr, d/ds, d/dt) of psi_ijk by the chain rule through (a,b,c), with the factors
    (1-b) and (1-c) cancelled analytically so the result is finite on the collapsed lines."""
    a, b, c = _rst_to_abc(r, s, t)
    C = 2.0 * math.sqrt(2.0)
    fa = jacobi_normalized(a, 0, 0, i)
    dfa = jacobi_normalized_deriv(a, 0, 0, i)
    gb = jacobi_normalized(b, 2 * i + 1, 0, j)
    dgb = jacobi_normalized_deriv(b, 2 * i + 1, 0, j)
    hc = jacobi_normalized(c, 2 * i + 2 * j + 2, 0, k)
    dhc = jacobi_normalized_deriv(c, 2 * i + 2 * j + 2, 0, k)
    ob, oc = 1.0 - b, 1.0 - c
    # common pieces
    t_a = dfa * gb * _pw(ob, i - 1) * hc * _pw(oc, i + j - 1)          # from d/da
    t_b = fa * (dgb * _pw(ob, i) - i * gb * _pw(ob, i - 1)) * hc * _pw(oc, i + j - 1)  # from d/db
    t_c = fa * gb * _pw(ob, i) * (dhc * _pw(oc, i + j) - (i + j) * hc * _pw(oc, i + j - 1))
    dr = 4.0 * C * t_a
    ds = 2.0 * C * (1.0 + a) * t_a + 2.0 * C * t_b
    dt = 2.0 * C * (1.0 + a) * t_a + C * (1.0 + b) * t_b + C * t_c
    return dr, ds, dt


def basis2d(r, s, i, j):
    """Orthonormal triangle basis sqrt2 P_i(a) P_j^(2i+1,0)(b) (1-b)^i, a = 2(1+r)/(1-s)-1, b=s."""
    a = np.full_like(r, -1.0)
    ok = np.abs(1.0 - s) > 1e-12
    a[ok] = 2.0 * (1.0 + r[ok]) / (1.0 - s[ok]) - 1.0
    return math.sqrt(2.0) * jacobi_normalized(a, 0, 0, i) * jacobi_normalized(s, 2 * i + 1, 0, j) * _pw(1.0 - s, i)


def vandermonde3d(N, rst):
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    return np.stack([basis3d(r, s, t, i, j, k) for (i, j, k) in basis_modes(N)], axis=1)


def grad_vandermonde3d(N, rst):
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    cols = [grad_basis3d(r, s, t, i, j, k) for (i, j, k) in basis_modes(N)]
    return (np.stack([c[0] for c in cols], axis=1), np.stack([c[1] for c in cols], axis=1),
            np.stack([c[2] for c in cols], axis=1))


def vandermonde2d(N, rs):
    modes = [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]
    return np.stack([basis2d(rs[:, 0], rs[:, 1], i, j) for (i, j) in modes], axis=1)


# ----------------------------------------------------------------------------------------
# operators

class RefElement:
    """Reference operators for order N, all FP64.

    Attributes: N, Np, Nfp, rst (Np,3), V, Vr, Vs, Vt, M (mass), Dr, Ds, Dt (Np,Np),
    Fmask (4,Nfp), Emat (Np, 4 Nfp) embedded face masses, LIFT = M^-1 Emat.
    """

    def __init__(self, N: int):
        if N < 1:
            raise ValueError("order must be >= 1")
        self.N = N
        self.Np, self.Nfp = counts(N)
        self.rst = nodes(N)
        self.V = vandermonde3d(N, self.rst)
        self.Vr, self.Vs, self.Vt = grad_vandermonde3d(N, self.rst)
        vinv = np.linalg.inv(self.V)
        self.M = np.linalg.inv(self.V @ self.V.T)
        self.Dr = self.Vr @ vinv
        self.Ds = self.Vs @ vinv
        self.Dt = self.Vt @ vinv
        self.Fmask = face_masks(N)
        r, s, t = self.rst[:, 0], self.rst[:, 1], self.rst[:, 2]
        # in-face coordinates: (r,s) on F1, (r,t) on F2, (s,t) on F3 and F4
        face_coords = [(r, s), (r, t), (s, t), (s, t)]
        E = np.zeros((self.Np, 4 * self.Nfp))
        for f in range(4):
            fm = self.Fmask[f]
            c1, c2 = face_coords[f]
            V2 = vandermonde2d(N, np.stack([c1[fm], c2[fm]], axis=1))
            mf = np.linalg.inv(V2 @ V2.T)
            E[np.ix_(fm, np.arange(f * self.Nfp, (f + 1) * self.Nfp))] = mf
        self.Emat = E
        self.LIFT = self.V @ (self.V.T @ E)


@lru_cache(maxsize=None)
def ref_element(N: int) -> RefElement:
    return RefElement(N)

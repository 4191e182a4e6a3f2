"""Oracle mesh quantities (test infrastructure only; never part of the product path).

Sec. 2 (eq. dg-reference-matrices): every element is the image of the reference tetrahedron
under an affine map Psi_k, so the global operators are the reference ones combined with the
constant Jacobian J_k and the constant derivatives of the inverse map. Sec. 2.1: the facial
values entering the numerical flux are picked out of the volume nodes of the element (u^-)
and of the element across the face (u^+).

This module computes, in FP64 and by plain definitions:
  orientation fix (a negative Jacobian swaps local vertices 3 and 4),
  face connectivity by matching sorted global vertex triples,
  geometric factors rx..tz and J from the 3x3 affine Jacobian,
  outward unit normals, surface Jacobians sJ and Fscale = sJ/J,
  physical node coordinates,
  face-node maps vmapM / vmapP by nearest physical coordinate (the builder of the product
  derives them combinatorially instead; the two must agree exactly).
"""
from __future__ import annotations

import numpy as np

from .refelem import FACE_VERTS, RefElement


class MeshError(ValueError):
    pass


def element_vertices(vxyz, etov):
    """(K, 4, 3) vertex coordinates."""
    return np.asarray(vxyz, dtype=np.float64)[np.asarray(etov)]


def orient(vxyz, etov):
    """Return a copy of etov in which every element has a positive Jacobian: elements whose
    det[v2-v1, v3-v1, v4-v1] is negative get local vertices 3 and 4 (1-based) swapped.
    A zero determinant is a degenerate element and raises MeshError."""
    etov = np.array(etov, dtype=np.int64, copy=True)
    v = element_vertices(vxyz, etov)
    det = np.linalg.det(np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]], axis=2))
    if np.any(det == 0.0):
        raise MeshError("degenerate element")
    neg = det < 0
    etov[neg, 2], etov[neg, 3] = etov[neg, 3].copy(), etov[neg, 2].copy()
    return etov


def connect(etov):
    """Face connectivity (EToE, EToF), each (K, 4). A face whose sorted global vertex triple
    is shared with no other face is a boundary face and points to itself. More than two
    faces with one triple is a non-conforming mesh and raises MeshError."""
    etov = np.asarray(etov, dtype=np.int64)
    K = etov.shape[0]
    keys = np.stack([np.sort(etov[:, list(fv)], axis=1) for fv in FACE_VERTS], axis=1)  # K,4,3
    keys = keys.reshape(-1, 3)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    sk = keys[order]
    same_next = np.all(sk[1:] == sk[:-1], axis=1)
    if np.any(same_next[1:] & same_next[:-1]):
        raise MeshError("more than two faces share one vertex triple")
    EToE = np.repeat(np.arange(K)[:, None], 4, axis=1).ravel()
    EToF = np.tile(np.arange(4), K)
    idx = np.nonzero(same_next)[0]
    a, b = order[idx], order[idx + 1]
    EToE_new = EToE.copy()
    EToF_new = EToF.copy()
    EToE_new[a], EToF_new[a] = EToE[b], EToF[b]
    EToE_new[b], EToF_new[b] = EToE[a], EToF[a]
    return EToE_new.reshape(K, 4), EToF_new.reshape(K, 4)


def geometric_factors(vxyz, etov):
    """Per element: J (K,) and the inverse-map derivatives G (K, 3, 3) with
    G[k, mu, nu] = d r_mu / d x_nu, i.e. rows (rx,ry,rz), (sx,sy,sz), (tx,ty,tz).

    x(r,s,t) = 1/2 (-(1+r+s+t) v1 + (1+r) v2 + (1+s) v3 + (1+t) v4), so
    x_r = (v2-v1)/2, x_s = (v3-v1)/2, x_t = (v4-v1)/2, J = det[x_r x_s x_t].
    """
    v = element_vertices(vxyz, etov)
    A = np.stack([(v[:, 1] - v[:, 0]) / 2, (v[:, 2] - v[:, 0]) / 2, (v[:, 3] - v[:, 0]) / 2], axis=2)
    J = np.linalg.det(A)
    G = np.linalg.inv(A)
    return J, G


def normals(J, G):
    """Outward unit normals n (K,4,3), sJ (K,4) and Fscale = sJ/J (K,4).

    Unnormalised outward normals: F1 -grad t, F2 -grad s, F3 grad(r+s+t), F4 -grad r;
    sJ = |n~| J is the ratio of physical face area to the area of the face's projection onto
    its in-face reference coordinates.
    """
    gr, gs, gt = G[:, 0, :], G[:, 1, :], G[:, 2, :]
    nt = np.stack([-gt, -gs, gr + gs + gt, -gr], axis=1)
    mag = np.linalg.norm(nt, axis=2)
    n = nt / mag[:, :, None]
    sJ = mag * J[:, None]
    return n, sJ, sJ / J[:, None]


def physical_nodes(vxyz, etov, rst):
    """Node coordinates (3, K, Np)."""
    v = element_vertices(vxyz, etov)
    r, s, t = rst[:, 0], rst[:, 1], rst[:, 2]
    w = np.stack([-(1 + r + s + t), 1 + r, 1 + s, 1 + t], axis=0) / 2.0  # 4, Np
    return np.einsum("vn,kvd->dkn", w, v)


def face_maps(x, EToE, EToF, Fmask, elems=None, hrel_match=1e-9, hrel_sep=1e-3):
    """vmapM, vmapP of shape (len(elems), 4, Nfp) with flat node ids k*Np + n.

    vmapP is found by nearest physical coordinate among the neighbour face's nodes; the
    nearest must be within hrel_match*h and the second nearest farther than hrel_sep*h
    (h the diameter of the face), else MeshError. Boundary faces map to themselves.
    Work is done in chunks of elements to bound memory.
    """
    _, K, Np = x.shape
    Nfp = Fmask.shape[1]
    if elems is None:
        elems = np.arange(K)
    elems = np.asarray(elems, dtype=np.int64)
    vM = elems[:, None, None] * Np + Fmask[None, :, :]
    vP = vM.copy()
    pts = np.transpose(x, (1, 2, 0))  # K, Np, 3
    chunk = 16384
    if elems.size > chunk:
        outM, outP = [], []
        for c0 in range(0, elems.size, chunk):
            a, b = face_maps(x, EToE, EToF, Fmask, elems[c0:c0 + chunk], hrel_match, hrel_sep)
            outM.append(a)
            outP.append(b)
        return np.concatenate(outM), np.concatenate(outP)
    for f in range(4):
        nb = EToE[elems, f]
        nf = EToF[elems, f]
        interior = (nb != elems) | (nf != f)
        ids = np.nonzero(interior)[0]
        if ids.size == 0:
            continue
        k = elems[ids]
        mine = pts[k][:, Fmask[f], :]                                  # m, Nfp, 3
        theirs = pts[nb[ids][:, None], Fmask[nf[ids]], :]               # m, Nfp, 3
        d = np.linalg.norm(mine[:, :, None, :] - theirs[:, None, :, :], axis=3)  # m,Nfp,Nfp
        hk = np.max(np.linalg.norm(pts[k][:, Fmask[f][:, None], :] - pts[k][:, Fmask[f][None, :], :],
                                   axis=3), axis=(1, 2))
        if Nfp > 1:
            srt = np.sort(d, axis=2)
            if np.any(srt[:, :, 0] > hrel_match * hk[:, None]) or np.any(srt[:, :, 1] < hrel_sep * hk[:, None]):
                raise MeshError("face nodes do not match")
        j = np.argmin(d, axis=2)
        vP[ids, f, :] = nb[ids][:, None] * Np + Fmask[nf[ids]][np.arange(ids.size)[:, None], j]
    return vM, vP


class Mesh:
    """All oracle mesh data for one (vxyz, etov) at order N."""

    def __init__(self, vxyz, etov, ref: RefElement, compute_maps=True):
        self.ref = ref
        self.vxyz = np.asarray(vxyz, dtype=np.float64)
        self.etov = orient(self.vxyz, etov)
        self.K = self.etov.shape[0]
        self.EToE, self.EToF = connect(self.etov)
        self.J, self.G = geometric_factors(self.vxyz, self.etov)
        if np.any(self.J <= 0):
            raise MeshError("non-positive Jacobian")
        self.n, self.sJ, self.Fscale = normals(self.J, self.G)
        self.x = physical_nodes(self.vxyz, self.etov, ref.rst)
        self.boundary = (self.EToE == np.arange(self.K)[:, None]) & (self.EToF == np.arange(4)[None, :])
        if compute_maps:
            self.vmapM, self.vmapP = face_maps(self.x, self.EToE, self.EToF, ref.Fmask)

"""Seeded synthetic inputs shared by the oracle tests, the GPU parity tests and the benchmark.

This module holds no arithmetic of the DG method itself: it only writes meshes (vertex
coordinates and element-to-vertex tables), draws random numbers, and evaluates closed-form
input functions at points the caller supplies.

Meshes stand in for the TetGen meshes of the paper's experiments (Sec. 6): a unit cube split
into n^3 small cubes, each cut into the six Kuhn tetrahedra sharing the main diagonal. The
perfectly conducting cavity test of Sec. 6 is represented by the (1,1,0) TM mode of the unit
cube, whose closed form is given by `cavity_tm110`.

Seeds (NumPy PCG64): jitter 1, element permutation 2, smooth fields 3, batch 4, arrivals 5,
materials 6, local vertex order 7.
"""
from __future__ import annotations

import math
from itertools import permutations

import numpy as np

SEED_JITTER = 1
SEED_PERM = 2
SEED_FIELDS = 3
SEED_BATCH = 4
SEED_ARRIVALS = 5
SEED_MATERIAL = 6
SEED_SHUFFLE = 7

# Vertex triples of the four faces of a tetrahedron (v1..v4 = 0..3), the numbering of the
# library interface: F1 = (v1,v2,v3), F2 = (v1,v2,v4), F3 = (v2,v3,v4), F4 = (v1,v3,v4).
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))

# Axis orders (x=0, y=1, z=2) in lexicographic order; the Kuhn tetrahedron p walks the cube
# diagonal along these axes.
_AXIS_ORDERS = list(permutations(range(3)))
# Odd permutations get their last two vertices swapped so every tetrahedron is positively
# oriented.
_ODD = {1, 2, 5}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def kuhn_cube(n: int, jitter: float = 0.0, permute: bool = False,
              seed_jitter: int = SEED_JITTER, seed_perm: int = SEED_PERM,
              nx: int | None = None, ny: int | None = None, nz: int | None = None,
              shuffle: bool = False, seed_shuffle: int = SEED_SHUFFLE):
    """Unit-cube tetrahedral mesh of 6*nx*ny*nz Kuhn tetrahedra.

    Returns (vxyz, etov): vxyz is (nverts, 3) float64, etov is (K, 4) int32, 0-based.
    Vertex id = (iz*(ny+1) + iy)*(nx+1) + ix at (ix/nx, iy/ny, iz/nz).
    Element id = ((cz*ny + cy)*nx + cx)*6 + p before the optional permutation.
    `jitter` moves every interior vertex by U(-jitter*h, jitter*h) per coordinate, with h the
    cell width along that axis; `permute` shuffles the element order (Fisher-Yates);
    `shuffle` lists the four vertices of every element in a random order of its own (half of
    the elements then come out negatively oriented), so that neighbouring elements meet in
    every relative face numbering and vertex rotation a conforming mesh allows.
    """
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    ix, iy, iz = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                             indexing="ij")
    # vertex id order: ix fastest, then iy, then iz
    ix = ix.transpose(2, 1, 0).ravel()
    iy = iy.transpose(2, 1, 0).ravel()
    iz = iz.transpose(2, 1, 0).ravel()
    vxyz = np.stack([ix / nx, iy / ny, iz / nz], axis=1).astype(np.float64)

    def vid(cx, cy, cz):
        return (cz * (ny + 1) + cy) * (nx + 1) + cx

    cx, cy, cz = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    cx = cx.transpose(2, 1, 0).ravel()
    cy = cy.transpose(2, 1, 0).ravel()
    cz = cz.transpose(2, 1, 0).ravel()
    ncell = cx.size
    etov = np.empty((ncell, 6, 4), dtype=np.int64)
    for p, order in enumerate(_AXIS_ORDERS):
        c = np.stack([cx, cy, cz], axis=1)
        step1 = np.zeros(3, dtype=np.int64)
        step1[order[0]] = 1
        step2 = step1.copy()
        step2[order[1]] = 1
        corners = [c, c + step1, c + step2, c + 1]
        ids = [vid(q[:, 0], q[:, 1], q[:, 2]) for q in corners]
        if p in _ODD:
            ids[2], ids[3] = ids[3], ids[2]
        etov[:, p, :] = np.stack(ids, axis=1)
    etov = etov.reshape(-1, 4)

    if jitter > 0.0:
        g = rng(seed_jitter)
        h = np.array([1.0 / nx, 1.0 / ny, 1.0 / nz])
        off = g.uniform(-1.0, 1.0, size=vxyz.shape) * (jitter * h)
        interior = ((ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz))
        vxyz = vxyz + off * interior[:, None]
    if permute:
        g = rng(seed_perm)
        perm = g.permutation(etov.shape[0])
        etov = etov[perm]
    if shuffle:
        g = rng(seed_shuffle)
        order = np.argsort(g.random(etov.shape), axis=1)
        etov = np.take_along_axis(etov, order, axis=1)
    return vxyz, etov.astype(np.int32)


def smooth_field_modes(seed: int = SEED_FIELDS, nmodes: int = 8):
    """Parameters of six random smooth fields u_f = sum_m A_fm sin(pi k_fm . x + phi_fm).

    k_fm is drawn from {-3..3}^3 without the zero vector, A ~ U(-1,1), phi ~ U(0, 2 pi).
    Returns a dict of arrays k (6, nmodes, 3) int, amp (6, nmodes), phase (6, nmodes).
    """
    g = rng(seed)
    k = np.zeros((6, nmodes, 3), dtype=np.int64)
    for f in range(6):
        for m in range(nmodes):
            while True:
                cand = g.integers(-3, 4, size=3)
                if np.any(cand != 0):
                    break
            k[f, m] = cand
    amp = g.uniform(-1.0, 1.0, size=(6, nmodes))
    phase = g.uniform(0.0, 2.0 * math.pi, size=(6, nmodes))
    return {"k": k, "amp": amp, "phase": phase}


def eval_smooth_fields(modes, x, y, z):
    """Evaluate the six random smooth fields at points (x, y, z) of any common shape.

    Returns an array of shape (6,) + x.shape, float64.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    out = np.zeros((6,) + x.shape, dtype=np.float64)
    k, amp, phase = modes["k"], modes["amp"], modes["phase"]
    for f in range(6):
        for m in range(k.shape[1]):
            arg = math.pi * (k[f, m, 0] * x + k[f, m, 1] * y + k[f, m, 2] * z) + phase[f, m]
            out[f] += amp[f, m] * np.sin(arg)
    return out


def cavity_tm110(x, y, z, t: float, eps: float = 1.0, mu: float = 1.0):
    """(1,1,0) TM eigenmode of the perfectly conducting unit-cube cavity filled with a uniform
    medium (default vacuum, eps = mu = 1).

    E = (0, 0, sin(pi x) sin(pi y) cos(w t)),  w = pi sqrt(2) / sqrt(eps mu),
    H = (1/(Z w')) (-pi sin(pi x) cos(pi y), pi cos(pi x) sin(pi y), 0) sin(w t),
    with Z = sqrt(mu/eps) and w' = pi sqrt(2) (it solves eps E_t = curl H, mu H_t = -curl E).
    Returns (6,) + x.shape float64 in the order Ex, Ey, Ez, Hx, Hy, Hz.
    """
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    w0 = math.pi * math.sqrt(2.0)
    w = w0 / math.sqrt(eps * mu)
    zi = math.sqrt(eps / mu)          # 1 / Z
    out = np.zeros((6,) + x.shape, dtype=np.float64)
    sx, cx = np.sin(math.pi * x), np.cos(math.pi * x)
    sy, cy = np.sin(math.pi * y), np.cos(math.pi * y)
    out[2] = sx * sy * math.cos(w * t)
    out[3] = -zi * (math.pi / w0) * sx * cy * math.sin(w * t)
    out[4] = zi * (math.pi / w0) * cx * sy * math.sin(w * t)
    return out


def random_materials(K: int, seed: int = SEED_MATERIAL, lo: float = 1.0, hi: float = 4.0):
    """Piecewise-constant permittivity and permeability, one value per element,
    log-uniform in [lo, hi] (independent draws for eps and mu)."""
    g = np.random.Generator(np.random.PCG64(seed))
    eps = np.exp(g.uniform(math.log(lo), math.log(hi), K))
    mu = np.exp(g.uniform(math.log(lo), math.log(hi), K))
    return eps, mu


def faces_on_plane(vxyz, etov, axis: int, value: float, tol: float = 1e-12):
    """(K, 4) int8 mask of the element faces lying in the plane x_axis = value; face f of
    element k is the vertex triple FACE_VERTS[f] of etov[k] as given."""
    vxyz = np.asarray(vxyz, dtype=np.float64)
    etov = np.asarray(etov)
    on = np.abs(vxyz[:, axis] - value) <= tol
    mask = np.zeros(etov.shape, dtype=np.int8)
    for f, tri in enumerate(FACE_VERTS):
        mask[:, f] = np.all(on[etov[:, list(tri)]], axis=1)
    return mask


def batch_specs(count: int = 64, seed: int = SEED_BATCH, kmin: float = 1e3, kmax: float = 5e4,
                nmin: int = 2, nmax: int = 6):
    """Mesh sizes and orders of a batch of independent cube meshes.

    K_target ~ logU[kmin, kmax]; nx = ny = floor((K/6)^(1/3)), nz = max(1, round(K/(6 nx ny)));
    N ~ U{nmin..nmax}. Returns a list of dicts with keys nx, ny, nz, order.
    """
    g = rng(seed)
    out = []
    for _ in range(count):
        kt = math.exp(g.uniform(math.log(kmin), math.log(kmax)))
        nx = max(1, int(math.floor((kt / 6.0) ** (1.0 / 3.0))))
        nz = max(1, int(round(kt / (6.0 * nx * nx))))
        order = int(g.integers(nmin, nmax + 1))
        out.append({"nx": nx, "ny": nx, "nz": nz, "order": order})
    return out

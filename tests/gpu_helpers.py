"""Helpers shared by the GPU tests: run the library through its binding and compare with the
oracle on the same seeded inputs."""
import sys

import numpy as np

import dginputs
import paper_0901_1024_amd as P
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm((np.asarray(a, np.float64) - b).ravel()) / np.linalg.norm(np.ravel(b)))


def per_field_rel(a, b):
    """Per-field error normalised by the norm of the whole state (fields may vanish)."""
    tot = np.linalg.norm(np.ravel(b))
    return [float(np.linalg.norm((np.asarray(a[f], np.float64) - b[f]).ravel()) / tot) for f in range(6)]


def gpu_rhs(solver, u):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(u, dtype=solver.dtype)).cuda()
    out = torch.empty_like(t)
    solver.rhs(t, out)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def problem(N, n, jitter=0.0, permute=False, fields="smooth", compute_maps=True):
    """Oracle mesh and initial fields for an n^3 Kuhn cube at order N."""
    v, e = dginputs.kuhn_cube(n, jitter=jitter, permute=permute)
    m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=compute_maps)
    x, y, z = m.x
    if fields == "cavity":
        u = dginputs.cavity_tm110(x, y, z, 0.0)
    else:
        u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x, y, z)
    return v, e, m, u


def rounded(u, prec):
    """The input as the device sees it, back in FP64 (input rounding is not charged)."""
    return np.asarray(u, dtype=np.float32).astype(np.float64) if prec == "f32" else np.asarray(u, np.float64)


def face_combos(vxyz, etov):
    """Distinct (face, neighbour face, vertex permutation) triples over the interior faces of a
    mesh, from the oracle's orientation fix and connectivity: the permutation p has my face
    vertex a equal to the neighbour's face vertex p[a]. Conforming, positively oriented
    tetrahedra allow 48 of the 96 triples."""
    et = Mm.orient(vxyz, etov)
    e2e, e2f = Mm.connect(et)
    fv = R.FACE_VERTS
    out = set()
    for k in range(et.shape[0]):
        for f in range(4):
            k2, f2 = int(e2e[k, f]), int(e2f[k, f])
            if k2 == k and f2 == f:
                continue
            mine = [int(et[k][fv[f][a]]) for a in range(3)]
            theirs = [int(et[k2][fv[f2][a]]) for a in range(3)]
            out.add((f, f2, tuple(theirs.index(x) for x in mine)))
    return out


def max_rel(a, b):
    """Largest pointwise difference relative to the largest reference value: a wrong face or
    element shows up here even when the global relative L2 dilutes it."""
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / np.max(np.abs(b)))


# pointwise bounds beside the relative L2 ones
MAX_TOL = {"f64": 1e-11, "f32": 1e-4}

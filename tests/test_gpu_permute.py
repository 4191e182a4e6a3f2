"""Canonical <-> internal permutes (dg_set_fields, dg_get_fields, dg_rhs) on the GPU.

The permutes move chunks of consecutive user elements through an LDS tile whose size depends on
the order and the precision (at most 64 elements and 32 KB). Checked here: bitwise round trips
of random fields at every order in both precisions, through the host and the device paths, on
meshes whose element count leaves a ragged last chunk; the right-hand side of dg_rhs against the
oracle on the same meshes; and a mesh with more chunks than the permute grid (8192 workgroups),
so that the grid-stride loop runs. Kuhn cubes have 6 n^3 elements, a multiple of the 3- and
6-element chunks of the highest orders, so the meshes here drop the cube's last element (its
neighbours' faces become walls): 749 elements leave a ragged last chunk at every order.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, gpu_rhs, max_rel, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def chunk(N, prec):
    """Elements per permute chunk: the LDS tile of 6 S words per element held to 32 KB."""
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    S = (Np + 3) // 4 * 4 if prec == "f32" and 3 <= N <= 7 else Np
    ce = 32768 // (6 * S * (8 if prec == "f64" else 4))
    return min(64, max(1, ce))


def round_trip(s, prec, seed):
    import torch
    g = np.random.default_rng(seed)
    u = g.standard_normal((6, s.K, s.Np)).astype(s.dtype)
    s.set_fields(u)
    assert np.array_equal(s.get_fields(), u)
    t = torch.from_numpy(u[::-1].copy()).cuda()
    s.set_fields(t)
    back = torch.empty_like(t)
    s.get_fields(back)
    torch.cuda.synchronize()
    assert torch.equal(back, t)


@pytest.mark.parametrize("N", range(1, 10))
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_round_trip_and_rhs_with_a_ragged_last_chunk(prec, N):
    ce = chunk(N, prec)
    v, e = dginputs.kuhn_cube(5, jitter=0.15, permute=True)
    e = e[:-1]
    assert e.shape[0] % ce
    say(f"case: permutes N={N} {prec} K={e.shape[0]} chunk {ce} (last chunk {e.shape[0] % ce})")
    s = P.Solver(v, e, N, prec, reorder=1)
    round_trip(s, prec, seed=N)
    m = Mm.Mesh(v, e, R.ref_element(N))
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), prec)
    r, ro = gpu_rhs(s, u), W.rhs(m, u)
    assert rel_l2(r, ro) <= TOL[prec] and max_rel(r, ro) <= MAX_TOL[prec]
    s.free()


def test_round_trip_with_more_chunks_than_the_grid():
    # FP64 N = 9: 3 elements per chunk, 6 * 17^3 - 1 = 29,477 elements = 9,826 chunks > 8,192
    N, prec, n = 9, "f64", 17
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
    e = e[:-1]
    assert -(-e.shape[0] // chunk(N, prec)) > 8192
    say(f"case: permutes N={N} {prec} K={e.shape[0]} grid-stride")
    s = P.Solver(v, e, N, prec, reorder=1)
    round_trip(s, prec, seed=99)
    s.free()

"""Handle groups (dg_group_*) and the mixed-order batch on the GPU.

- A group of handles of different orders, precisions and kernels advanced from one captured
  graph equals each handle advanced alone, bitwise (same kernels, same arithmetic), also over
  odd step counts and repeated calls (graph replay);
- a batch of meshes of mixed orders (2..6, one batch handle per order, all in one group) takes
  its steps at each mesh's own stable step and matches the oracle mesh by mesh.
"""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, max_rel, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu


def _fields(s):
    x = s.nodes()
    return dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x[0], x[1], x[2]).astype(s.dtype)


def test_group_equals_members_alone():
    v, e = dginputs.kuhn_cube(4, jitter=0.15, permute=True)
    specs = [(2, "f32"), (3, "f64"), (4, "f32"), (5, "bf16x3"), (6, "f32")]
    grp, alone = [], []
    for N, prec in specs:
        a = P.Solver(v, e, N, prec)
        b = P.Solver(v, e, N, prec)
        u = _fields(a)
        a.set_fields(u)
        b.set_fields(u)
        grp.append(a)
        alone.append(b)
    dts = [s.stable_dt() for s in grp]
    g = P.Group(grp)
    for n in (4, 3, 6):
        say(f"case: group of {len(grp)} members, {n} steps")
        g.solve(dts, n)
        for s, dt in zip(alone, dts):
            s.solve(dt, n)
        for (N, prec), a, b in zip(specs, grp, alone):
            assert np.array_equal(a.get_fields(), b.get_fields()), (N, prec)
            assert a.time == b.time
    g.free()
    for s in grp + alone:
        s.free()


def test_mixed_order_batch_matches_oracle():
    g = np.random.default_rng(4)
    meshes, orders, oms = [], [], []
    for i, (n, N) in enumerate([(2, 2), (3, 4), (2, 6), (3, 3), (2, 5), (3, 2)]):
        v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True, shuffle=True, seed_jitter=80 + i,
                                  seed_perm=90 + i)
        md = {"vxyz": v, "etov": e}
        m = Mm.Mesh(v, e, R.ref_element(N))
        kw = {}
        if i == 1:      # one mesh in a medium with absorbing faces
            md["eps"], md["mu"] = dginputs.random_materials(e.shape[0], seed=91)
            md["face_bc"] = dginputs.faces_on_plane(v, e, 2, 1.0) * 2
            kw = dict(eps=md["eps"], mu=md["mu"], absorb=dginputs.faces_on_plane(v, m.etov, 2, 1.0).astype(bool))
        meshes.append(md)
        orders.append(N)
        oms.append((m, kw))
    mb = P.MixedBatch(meshes, orders, "f32")
    say(f"case: mixed-order batch, orders {mb.orders}, K={mb.K}")
    us = [rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), "f32") for m, _ in oms]
    dts = mb.stable_dts(0.5)
    mb.set_dts(dts)
    mb.set_fields(us)
    mb.solve(3)
    got = mb.get_fields()
    for i, ((m, kw), u) in enumerate(zip(oms, us)):
        uo, res = u, None
        for _ in range(3):
            uo, res = W.lsrk4_step(m, uo, dts[i], res=res, **kw)
        err, mx = rel_l2(got[i], uo), max_rel(got[i], uo)
        say(f"  mesh {i}: N={orders[i]} K={m.K} dt={dts[i]:.3e} 3 steps rel {err:.2e} max {mx:.2e}")
        assert err <= 1e-5 and mx <= MAX_TOL["f32"], i
    mb.free()

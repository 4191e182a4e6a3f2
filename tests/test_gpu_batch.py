"""The batched form on the GPU: one handle holding several meshes (different K, geometry,
face conditions, materials) equals one handle per mesh. On the element-wise kernel (FP64 N = 2)
the right-hand side is bitwise equal (its per-element arithmetic does not depend on the
element's position); a contraction kernel may round an element's face fluxes differently at
another position in its tile, so there the bound is 1e-6 in FP32 and 1e-13 in FP64 (N = 5 on
the FP64 high-order kernel). RK steps with per-mesh time steps agree to the parity tolerances
(the step is folded into the geometric records, which changes the rounding, not the
operator)."""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import gpu_rhs, rel_l2, rounded, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def batch_meshes(prec):
    out = []
    for i, (n, jit) in enumerate([(2, 0.0), (3, 0.15), (1, 0.1), (3, 0.1)]):
        v, e = dginputs.kuhn_cube(n, jitter=jit, permute=True)
        md = {"vxyz": v, "etov": e}
        if i == 3:
            md["eps"], md["mu"] = dginputs.random_materials(e.shape[0], seed=31)
            md["face_bc"] = dginputs.faces_on_plane(v, e, 2, 1.0) * 2
        out.append(md)
    return out


@pytest.mark.parametrize("prec,N", [("f64", 2), ("f64", 5), ("f32", 3), ("f32", 4), ("f32", 5)])
def test_batch_equals_one_handle_per_mesh(prec, N):
    say(f"case: batch of 4 meshes N={N} {prec}")
    meshes = batch_meshes(prec)
    b = P.BatchSolver(meshes, N, prec)
    singles = [P.Solver(md["vxyz"], md["etov"], N, prec, face_bc=md.get("face_bc"),
                        eps=md.get("eps"), mu=md.get("mu")) for md in meshes]
    us = [rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *s.nodes()), prec)
          for s in singles]
    ub = np.concatenate(us, axis=1)
    rb = gpu_rhs(b, ub)
    for i, s in enumerate(singles):
        r1 = gpu_rhs(s, us[i])
        if prec == "f64" and N == 2:
            assert np.array_equal(rb[:, b.mesh_slice(i)], r1)
        else:
            assert rel_l2(rb[:, b.mesh_slice(i)], r1) <= (1e-13 if prec == "f64" else 1e-6)
    dts = b.stable_dts(0.5)
    b.set_dts(dts)
    b.set_fields(ub)
    eb = b.energy()
    b.solve(1.0, 5)                     # two graph replays and one plain step, all meshes
    got = b.get_fields()
    e_single = 0.0
    for i, s in enumerate(singles):
        s.set_fields(us[i])
        e_single += s.energy()
        s.solve(dts[i], 5)
        err = rel_l2(got[:, b.mesh_slice(i)], s.get_fields())
        say(f"  mesh {i}: K={s.K} dt={dts[i]:.3e} rel {err:.2e}")
        assert err <= TOL[prec]
    assert abs(eb - e_single) <= 1e-12 * e_single


def test_batch_matches_the_oracle():
    meshes = batch_meshes("f64")[:3]
    b = P.BatchSolver(meshes, 3, "f64")
    dts = b.stable_dts(0.5)
    b.set_dts(dts)
    us, oms = [], []
    for md in meshes:
        m = Mm.Mesh(md["vxyz"], md["etov"], R.ref_element(3))
        oms.append(m)
        us.append(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x))
    b.set_fields(np.concatenate(us, axis=1))
    b.solve(1.0, 2)
    got = b.get_fields()
    for i, m in enumerate(oms):
        uo, res = us[i], None
        for _ in range(2):
            uo, res = W.lsrk4_step(m, uo, dts[i], res)
        assert rel_l2(got[:, b.mesh_slice(i)], uo) <= TOL["f64"]


def test_batch_time_step_errors():
    import ctypes
    meshes = batch_meshes("f32")[:2]
    b = P.BatchSolver(meshes, 3, "f32")
    with pytest.raises(P.DGError, match="DG_E_ARG"):
        b.set_dts(np.array([1e-3, -1.0]))
    with pytest.raises(P.DGError, match="DG_E_ARG"):
        b.set_dts(np.array([1e-3, np.nan]))
    with pytest.raises(P.DGError, match="DG_E_ARG"):
        b.set_dts(np.array([1e-3]))
    s = P.Solver(meshes[0]["vxyz"], meshes[0]["etov"], 3, "f32")
    d = np.array([1e-3])
    rc = P.lib().dg_set_batch_dt(s._h, d.ctypes.data_as(ctypes.c_void_p), None)
    assert rc == P.DG_E_ARG          # not a batch handle
    c = ctypes.c_int32()
    first = np.zeros(2, dtype=np.int32)
    assert P.lib().dg_batch_info(s._h, ctypes.byref(c), first.ctypes.data_as(ctypes.c_void_p)) == 0
    assert c.value == 1 and list(first) == [0, s.K]

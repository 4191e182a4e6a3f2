"""Kernel choice (dg_opts.tile_id) on the GPU: both kernel families of an order agree with the
oracle, and the autotuner's table is honoured."""
import json

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


@pytest.mark.parametrize("prec,N", [("f32", 3), ("f32", 5), ("f32", 6), ("f32", 7), ("f64", 3), ("f64", 4),
                                    ("f64", 5), ("f64", 6), ("f64", 7)])
def test_both_kernel_families_match_oracle(prec, N):
    v, e = dginputs.kuhn_cube(3, jitter=0.15, permute=True, shuffle=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    u = rounded(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x), prec)
    ro = W.rhs(m, u)
    dt = W.stable_dt(m)
    uo, _ = W.lsrk4_step(m, u, dt)
    for tid in (1, 2, 3) if (prec, N) == ("f32", 3) else (1, 2):
        say(f"case: tile_id {tid} {prec} N={N}")
        s = P.Solver(v, e, N, prec, tile_id=tid)
        r = gpu_rhs(s, u)
        assert rel_l2(r, ro) <= TOL[prec] and max_rel(r, ro) <= MAX_TOL[prec], tid
        s.set_fields(u)
        s.rk_step(dt)
        ug = s.get_fields()
        assert rel_l2(ug, uo) <= TOL[prec] and max_rel(ug, uo) <= MAX_TOL[prec], tid
        s.free()


def test_autotuner_table_is_honoured(tmp_path, monkeypatch):
    from paper_0901_1024_amd import tune
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"choices": {"f32/5": [{"K": 100, "tile_id": 1}, {"K": 100000, "tile_id": 2}]}}))
    monkeypatch.setenv("DG_TUNING_FILE", str(path))
    assert tune.choose(5, "f32", 120) == 1 and tune.choose(5, "f32", 50000) == 2
    assert tune.choose(4, "f32", 120) == 0            # no entry: library default
    v, e = dginputs.kuhn_cube(2)
    small = P.Solver(v, e, 5, "f32", tile_id="auto")
    big_default = P.Solver(v, e, 5, "f32")
    # the element-wise kernel needs no operator table: a smaller workspace
    assert small.workspace_bytes < big_default.workspace_bytes
    small.free()
    big_default.free()

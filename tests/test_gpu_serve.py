"""The serving loop on the GPU: every result is the same alone and in the mix (each solve's
arithmetic is independent of the others; it runs the same kernels on its own handle), and
every served result equals the FP64 oracle's LSRK4 solve of the same request (FP32
tolerances, the oracle starting from the FP32-rounded initial fields)."""
import numpy as np
import pytest

import dginputs
import paper_0901_1024_amd as P
from gpu_helpers import MAX_TOL, max_rel, rel_l2, say
from oracle import maxwell as W
from oracle import mesh as Mm
from oracle import refelem as R
from paper_0901_1024_amd.serve import Request, Server, summary

pytestmark = pytest.mark.gpu


def _cavity(x):
    return dginputs.cavity_tm110(x[0], x[1], x[2], 0.0)


def test_results_are_the_same_alone_and_in_the_mix():
    specs = [(2, 3, 10), (3, 4, 6), (2, 5, 8), (3, 3, 12), (1, 6, 4), (4, 4, 6), (2, 4, 10)]
    reqs = []
    for i, (n, N, steps) in enumerate(specs):
        v, e = dginputs.kuhn_cube(n, jitter=0.1, permute=True, seed_jitter=10 + i)
        reqs.append(Request(rid=i, arrival=0.002 * i, vxyz=v, etov=e, order=N, steps=steps,
                            init=_cavity))
    done = Server(budget_bytes=2 ** 30, slots=4, chunk_steps=4, keep_results=True).run(reqs)
    assert len(done) == len(specs)
    say("served:", summary(done))
    for r in done:
        s = P.Solver(r.vxyz, r.etov, r.order, "f32")
        s.set_fields(_cavity(s.nodes()).astype(np.float32))
        s.solve(s.stable_dt(0.5), r.steps)
        assert np.array_equal(s.get_fields(), r.result), r.rid
        # the FP64 oracle on the same request
        m = Mm.Mesh(r.vxyz, r.etov, R.ref_element(r.order))
        u = _cavity(m.x).astype(np.float32).astype(np.float64)
        dt = W.stable_dt(m)
        assert abs(dt - s.stable_dt(0.5)) <= 1e-14 * dt
        res = None
        for _ in range(r.steps):
            u, res = W.lsrk4_step(m, u, dt, res)
        err, mx = rel_l2(r.result, u), max_rel(r.result, u)
        say(f"  request {r.rid}: N={r.order} K={m.K} steps={r.steps} vs oracle rel {err:.2e} max {mx:.2e}")
        assert err <= 1e-5 and mx <= MAX_TOL["f32"], r.rid

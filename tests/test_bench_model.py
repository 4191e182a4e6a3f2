"""bench.py's work model and its one-GPU contract (CPU only).

The roofline's numerator is the algorithmic flop count of the right-hand side per element
(adds and multiplies, FMA = 2, no padding): reference derivatives 36 Np^2, combine and curl
66 Np, lift 48 Np Nfp + 6 Np, upwind flux 58 per face node. The expected values below were
tabulated independently (per order, from the operation counts of Sec. 5) before the benchmark
was written; the stage adds the RK update, 30 Np.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

RHS_FLOPS = {2: 8_592, 3: 27_760, 4: 75_300, 5: 178_248, 6: 379_456, 7: 742_752}


@pytest.mark.parametrize("N", sorted(RHS_FLOPS))
def test_rhs_flop_model_matches_the_tabulated_counts(N):
    Np, _ = bench.counts(N)
    assert bench.rhs_flops_per_elem(N) == RHS_FLOPS[N]
    assert bench.flops_per_elem_stage(N) == RHS_FLOPS[N] + 30 * Np


def test_compulsory_bytes_of_the_headline_stage():
    # FP32 N = 4: read u and res, write u and res (24 x 35 words), 25 geometry words, 16 B of
    # face records
    assert bench.bytes_per_elem_stage(4, 4) == 3_476
    assert bench.bytes_per_elem_stage(3, 8) == 4_056


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr

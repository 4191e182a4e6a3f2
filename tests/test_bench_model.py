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


def _traffic_file(dirpath, sha, value=1.5e9):
    prof = os.path.join(dirpath, "profiles")
    os.makedirs(prof, exist_ok=True)
    with open(os.path.join(prof, "stage_f32_n4_k384000_traffic.txt"), "w") as fh:
        fh.write("# HBM traffic of one launch\nkernel: mfma_stage_kernel<4, true, false, false>\n"
                 f"kernel_source_sha256: {sha}\ntraffic_bytes_per_launch: {value}\n")


def test_recorded_traffic_is_dropped_once_the_kernel_source_changes(tmp_path, monkeypatch):
    """The traffic of a committed counter summary is reported only for the kernel source it was
    measured on (its SHA-256); after any change to that source the bench line says null."""
    import hashlib
    src = tmp_path / "kernels.hip"
    src.write_bytes(b"// kernel source as profiled\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(src))
    _traffic_file(str(tmp_path), hashlib.sha256(src.read_bytes()).hexdigest())
    assert bench.recorded_traffic(4, "f32", 384000) == 1.5e9
    src.write_bytes(b"// kernel source as profiled, then edited\n")
    assert bench.recorded_traffic(4, "f32", 384000) is None
    assert bench.recorded_traffic(5, "f32", 196608) is None        # no summary for that workload


def test_committed_traffic_summaries_name_their_source_and_bytes():
    prof = os.path.join(ROOT, "profiles")
    names = [n for n in os.listdir(prof) if n.endswith("_traffic.txt")]
    assert names
    for n in names:
        rec = {}
        with open(os.path.join(prof, n)) as fh:
            for line in fh:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    rec[k.strip()] = v.strip()
        assert len(rec.get("kernel_source_sha256", "")) == 64, n
        assert float(rec["traffic_bytes_per_launch"]) > 0, n

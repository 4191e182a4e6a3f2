#!/usr/bin/env python3
"""Throughput of the nodal DG Maxwell hot path on one MI355X.

Workload: unit cube, 6 * 40^3 = 384,000 tetrahedra with interior vertices jittered by
+-0.15 h (seed 1) and elements randomly permuted (seed 2), order N = 4 (Np = 35), FP32,
perfectly conducting walls, six random smooth initial fields (seed 3). One step = one
five-stage low-storage RK4 step, i.e. five evaluations of the full semi-discrete operator
(volume curl, flux gather with the upwind flux and the wall mirror, lift) each fused with its
RK update. Timed: --steps steps after --warmup untimed ones, between HIP events on the
stream the kernels run on, inputs resident in HBM.

Prints one JSON line. `value` is algorithmic GFLOP/s (adds and multiplies, FMA = 2; no
padding work), the paper's measure of Sec. 6.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DG RHS GFLOP/s + HBM GB/s (roofline %); solves/s + p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0
# Dense peaks of the pipe each precision's contraction runs on. The split-BF16 form takes
# three bf16 products per FP32 product, so its peak in algorithmic (FP32-equivalent) flops is
# the bf16 matrix peak over three.
PEAKS_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16x3": 2500.0 / 3}


def counts(N):
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    Nfp = (N + 1) * (N + 2) // 2
    return Np, Nfp


def flops_per_elem_stage(N):
    """Algorithmic flops of one fused stage per element: reference derivatives 36 Np^2,
    physical combine + curl 66 Np, lift 48 Np Nfp + 6 Np, flux 58 per face node,
    RK update 5 per value."""
    Np, Nfp = counts(N)
    return 36 * Np * Np + 66 * Np + 48 * Np * Nfp + 6 * Np + 58 * 4 * Nfp + 30 * Np


def bytes_per_elem_stage(N, word, material=False):
    """Compulsory HBM bytes of one fused stage per element: read u and res, write u_out and
    res (24 Np words), the geometric record (9 + 16 words) and four face records (16 B); in a
    heterogeneous medium also the 20-word material record."""
    Np, _ = counts(N)
    return 24 * Np * word + 25 * word + 16 + (20 * word if material else 0)


KERNEL_SOURCE = os.path.join(ROOT, "paper_0901_1024_amd", "csrc", "kernels.hip")


def recorded_traffic(N, prec, K):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary of
    this workload, or None when the kernel source has changed since it was measured."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"stage_{prec}_n{N}_k{K}_traffic.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    with open(KERNEL_SOURCE, "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    if rec.get("kernel_source_sha256") != sha or "traffic_bytes_per_launch" not in rec:
        return None
    return float(rec["traffic_bytes_per_launch"])


def device_copy_gbs(torch, nbytes=1 << 30, reps=10):
    """Bytes moved (read + write) per second by torch's device-to-device copy of nbytes."""
    import numpy as np
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        t.append(e0.elapsed_time(e1) / 1e3)
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / float(np.median(t)) / 1e9


def rhs_flops_per_elem(N):
    """Algorithmic flops of one right-hand side per element (the fused stage without the
    30 Np of the RK update)."""
    Np, _ = counts(N)
    return flops_per_elem_stage(N) - 30 * Np


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


_POOL_STATE = {}


def _oracle_chunk(bounds):
    from oracle import maxwell as W
    m, u = _POOL_STATE["mesh"], _POOL_STATE["u"]
    return float(W.rhs_range(m, u, bounds[0], bounds[1])[0, 0, 0])


def cpu_baseline(N, n_sample, reps=5):
    """The FP64 oracle's right-hand side timed on the host cores, on a smaller mesh of the same
    recipe (jittered, permuted, smooth fields): one core (oracle.rhs, median of `reps` after a
    warm-up; the paper's comparison is one CPU core), and all cores of this process's affinity
    set (at most 16; the same arithmetic, oracle.rhs_range over disjoint element ranges in
    forked worker processes, median of `reps`). Plain NumPy loops, not a tuned BLAS code."""
    import multiprocessing as mp
    import statistics

    import dginputs
    from oracle import maxwell as W
    from oracle import mesh as Mm
    from oracle import refelem as R
    v, e = dginputs.kuhn_cube(n_sample, jitter=0.15, permute=True)
    m = Mm.Mesh(v, e, R.ref_element(N))
    u = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *m.x)
    flops = m.K * rhs_flops_per_elem(N)
    W.rhs(m, u)
    one = []
    for _ in range(reps):
        t0 = time.perf_counter()
        W.rhs(m, u)
        one.append(time.perf_counter() - t0)
    t1 = statistics.median(one)
    ncpu = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    workers = max(1, min(16, ncpu))
    _POOL_STATE["mesh"], _POOL_STATE["u"] = m, u
    chunk = (m.K + 4 * workers - 1) // (4 * workers)
    bounds = [(a, min(m.K, a + chunk)) for a in range(0, m.K, chunk)]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_chunk, bounds)            # warm-up
        alln = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pool.map(_oracle_chunk, bounds)
            alln.append(time.perf_counter() - t0)
    _POOL_STATE.clear()
    tall = statistics.median(alln)
    return {"value": round(flops / tall / 1e9, 3), "unit": "GFLOP/s", "cores": workers, "kind": "oracle",
            "sample": f"right-hand side of the FP64 NumPy oracle on 6*{n_sample}^3 = {m.K} jittered, permuted "
                      f"tets, N={N}, smooth fields; median of {reps} after a warm-up; all cores = {workers} "
                      f"forked workers over element ranges; a measured rate on this sample, not extrapolated",
            "seconds_per_rhs": round(tall, 4),
            "one_core": {"value": round(flops / t1 / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                         "seconds_per_rhs": round(t1, 4)},
            "host": {"nproc": os.cpu_count(), "affinity_cpus": ncpu, "cpu_model": cpu_model()}}


def run_batch(args):
    """Batched form: 64 independent jittered cube meshes (K log-uniform in [1e3, 5e4], N uniform
    in 2..6, FP32, seed 4), each advanced `batch_steps` steps with its own stable step. Plain:
    one handle per mesh, dg_solve mesh after mesh on one stream. Batched: one handle per order
    (all meshes of that order concatenated), dg_solve of each. Both start from the same fields,
    take two untimed warm-up steps, and must end within the FP32 parity tolerance."""
    import numpy as np
    import torch

    import dginputs
    import paper_0901_1024_amd as P

    specs = dginputs.batch_specs()
    meshes = []
    for i, sp in enumerate(specs):
        v, e = dginputs.kuhn_cube(0, jitter=0.15, permute=True, seed_jitter=100 + i, seed_perm=200 + i,
                                  nx=sp["nx"], ny=sp["ny"], nz=sp["nz"])
        meshes.append({"vxyz": v, "etov": e, "order": sp["order"]})
    steps, prec = args.batch_steps, "f32"
    plain = [P.Solver(md["vxyz"], md["etov"], md["order"], prec) for md in meshes]
    u0 = [dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), *s.nodes()) for s in plain]
    dts = [s.stable_dt(0.5) for s in plain]
    orders = sorted({md["order"] for md in meshes})
    groups = {N: [i for i, md in enumerate(meshes) if md["order"] == N] for N in orders}
    batched = {}
    for N, idx in groups.items():
        b = P.BatchSolver([meshes[i] for i in idx], N, prec)
        b.set_dts(b.stable_dts(0.5))
        b.set_fields(np.concatenate([u0[i] for i in idx], axis=1))
        batched[N] = b
    for i, s in enumerate(plain):
        s.set_fields(u0[i])
    stream = torch.cuda.current_stream()

    def timed(run):
        run(2)
        torch.cuda.synchronize()
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        run(steps)
        z.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(z) / 1e3

    t_plain = timed(lambda n: [s.solve(dts[i], n) for i, s in enumerate(plain)])
    t_orders = timed(lambda n: [b.solve(1.0, n) for b in batched.values()])
    # all orders from one captured graph (a group of the per-order batch handles); the handles
    # were advanced above, so the plain loop takes the same further steps for the comparison
    grp = P.Group(list(batched.values()))
    t_batch = timed(lambda n: grp.solve(np.ones(len(batched)), n))
    timed(lambda n: [s.solve(dts[i], n) for i, s in enumerate(plain)])
    # each order's graph on a stream of its own, joined on the timing stream
    streams = [torch.cuda.Stream() for _ in batched]

    def on_streams(n):
        ev = torch.cuda.Event()
        ev.record(stream)
        for st, b in zip(streams, batched.values()):
            st.wait_event(ev)
            b.solve(1.0, n, stream=st)
        for st in streams:
            stream.wait_stream(st)

    t_streams = timed(on_streams)
    timed(lambda n: [s.solve(dts[i], n) for i, s in enumerate(plain)])
    worst = 0.0
    for N, idx in groups.items():
        got = batched[N].get_fields()
        for j, i in enumerate(idx):
            ref = plain[i].get_fields()
            sl = batched[N].mesh_slice(j)
            worst = max(worst, float(np.linalg.norm(got[:, sl] - ref) / np.linalg.norm(ref)))
    if not worst <= 1e-5:
        print(f"batched and plain results differ: {worst:.2e}", file=sys.stderr)
        sys.exit(1)
    Ks = [md["etov"].shape[0] for md in meshes]
    flops = sum(5 * steps * K * flops_per_elem_stage(md["order"]) for K, md in zip(Ks, meshes))
    out = {
        "metric": "solves/s, batched (one handle per order, all orders in one graph) vs plain per-mesh loop",
        "value": round(len(meshes) / t_batch, 3), "unit": "solves/s", "n_gpus": 1, "steps": steps,
        "warmup": 2, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"64 jittered+permuted cube meshes, K log-uniform in [1e3, 5e4] "
                               f"(total {sum(Ks)}), N uniform in 2..6, FP32, {steps} steps each at "
                               f"its own stable step",
                   "meshes": len(meshes), "K_total": sum(Ks), "orders": {str(N): len(v) for N, v in groups.items()}},
        "plain_solves_per_s": round(len(meshes) / t_plain, 3),
        "speedup_batched_over_plain": round(t_plain / t_batch, 3),
        "batched_gflops": round(flops / t_batch / 1e9, 1), "plain_gflops": round(flops / t_plain / 1e9, 1),
        "seconds": {"batched": round(t_batch, 4), "plain": round(t_plain, 4),
                    "batched_one_graph_per_order": round(t_orders, 4),
                    "batched_one_stream_per_order": round(t_streams, 4)},
        "max_rel_diff_batched_vs_plain": worst,
    }
    for s_ in plain:
        s_.free()
    grp.free()
    for b in batched.values():
        b.free()
    return out


def run_serve(args, rates=(0.5, 1.0, 2.0)):
    """Serving form: cavity solves with K log-uniform in [2e3, 2e5], N uniform in 3..6, steps
    uniform in [100, 2000], FP32 (seed 5). Capacity = requests / makespan of the plain FIFO loop
    with everything queued at t = 0; then Poisson arrivals at 0.5, 1 and 2 times that rate,
    served with continuous admission (4 slots: the hardware queues a process gets; 64 GiB budget)
    and with the FIFO loop."""
    import math

    import numpy as np

    import dginputs
    from paper_0901_1024_amd.serve import Request, Server, summary

    g = np.random.Generator(np.random.PCG64(dginputs.SEED_ARRIVALS))
    specs = []
    for i in range(args.serve_requests):
        kt = math.exp(g.uniform(math.log(2e3), math.log(2e5)))
        nx = max(1, int(math.floor((kt / 6.0) ** (1.0 / 3.0))))
        nz = max(1, int(round(kt / (6.0 * nx * nx))))
        specs.append((nx, nz, int(g.integers(3, 7)), int(g.integers(100, 2001))))
    gaps = g.exponential(1.0, size=len(specs))

    def cavity(x):
        return dginputs.cavity_tm110(x[0], x[1], x[2], 0.0)

    meshes = [dginputs.kuhn_cube(0, jitter=0.15, permute=True, seed_jitter=300 + i, seed_perm=400 + i,
                                 nx=nx, ny=nx, nz=nz) for i, (nx, nz, _, _) in enumerate(specs)]

    def requests(rate):
        t = 0.0
        out = []
        for i, ((nx, nz, N, steps), (v, e)) in enumerate(zip(specs, meshes)):
            out.append(Request(rid=i, arrival=t, vxyz=v, etov=e, order=N, steps=steps, init=cavity))
            if rate:
                t += gaps[i] / rate
        return out

    budget = 64 * 2 ** 30
    fifo = lambda: Server(budget, slots=1, chunk_steps=args.serve_chunk)
    served = lambda: Server(budget, slots=args.serve_slots, chunk_steps=args.serve_chunk,
                            backfill=args.serve_backfill)
    base = summary(fifo().run(requests(0.0)))
    cap = base["solves_per_s"]
    print(f"capacity (FIFO, all queued): {cap:.3f} solves/s", file=sys.stderr, flush=True)
    sweep = []
    for mult in rates:
        rate = mult * cap
        a = summary(served().run(requests(rate)))
        b = summary(fifo().run(requests(rate)))
        print(f"rate {mult}x: served {a['solves_per_s']:.3f}/s p50 {a['p50_latency_s']:.3f} p99 "
              f"{a['p99_latency_s']:.3f} | fifo {b['solves_per_s']:.3f}/s p50 {b['p50_latency_s']:.3f} "
              f"p99 {b['p99_latency_s']:.3f}", file=sys.stderr, flush=True)
        sweep.append({"rate_x_capacity": mult, "arrival_rate": rate, "served": a, "fifo": b})
    top = sweep[-1]
    Ks = [6 * nx * nx * nz for nx, nz, _, _ in specs]
    out = {
        "metric": "solves/s + p50/p99 latency, continuous admission vs plain FIFO loop",
        "value": round(top["served"]["solves_per_s"], 3), "unit": "solves/s", "n_gpus": 1,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{len(specs)} cavity solves, K log-uniform in [2e3, 2e5] (total {sum(Ks)}), "
                               "N uniform in 3..6, steps uniform in [100, 2000], FP32, Poisson arrivals (seed 5)",
                   "slots": args.serve_slots, "chunk_steps": args.serve_chunk, "budget_bytes": budget,
                   "backfill": args.serve_backfill},
        "capacity_fifo_solves_per_s": cap,
        f"at_{rates[-1]:g}x_rate": {"served_p50_s": top["served"]["p50_latency_s"],
                                    "served_p99_s": top["served"]["p99_latency_s"],
                                    "fifo_solves_per_s": top["fifo"]["solves_per_s"],
                                    "fifo_p50_s": top["fifo"]["p50_latency_s"],
                                    "fifo_p99_s": top["fifo"]["p99_latency_s"]},
        "sweep": sweep,
    }
    return out


def run_precision_sweep(args):
    """Precision form: the (1,1,0) cavity mode on jittered cubes, run to t = T in FP64, FP32 and
    split-BF16 (the last at N = 5, 7) with the same step; per-field relative L2 difference
    against FP64, energy drift E(t)/E64(t) - 1, and the error of each against the exact mode.
    N = 7 runs to its own (shorter) time so that the FP64 leg, on the element-wise kernel at
    that order, stays within a few minutes."""
    import math

    import numpy as np
    import torch

    import dginputs
    import paper_0901_1024_amd as P
    from oracle import maxwell as W
    from oracle import mesh as Mm
    from oracle import refelem as R

    results = []
    for N, n, T in ((5, args.sweep_n5, args.sweep_t), (7, args.sweep_n7, args.sweep_t7)):
        v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
        m = Mm.Mesh(v, e, R.ref_element(N), compute_maps=False)
        u0 = dginputs.cavity_tm110(*m.x, 0.0)
        exact = dginputs.cavity_tm110(*m.x, T)
        row = {"order": N, "K": int(m.K), "t": T}
        fields = {}
        for prec in ("f64", "f32", "bf16x3"):
            s = P.Solver(v, e, N, prec)
            s.set_fields(u0.astype(s.dtype))
            dt0 = s.stable_dt(0.5)
            nsteps = int(math.ceil(T / dt0))
            dt = T / nsteps
            e0 = s.energy()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            done = 0
            while done < nsteps:
                k = min(500, nsteps - done)
                s.solve(dt, k)
                torch.cuda.synchronize()
                done += k
                print(f"  N={N} {prec}: {done}/{nsteps} steps", file=sys.stderr, flush=True)
            sec = time.perf_counter() - t0
            u = s.get_fields().astype(np.float64)
            fields[prec] = u
            err, nrm = W.l2_error(m, u, exact)
            flops = 5 * nsteps * m.K * flops_per_elem_stage(N)
            row[prec] = {"steps": nsteps, "dt": dt, "seconds": round(sec, 3),
                         "gflops": round(flops / sec / 1e9, 1), "energy_0": e0, "energy_T": s.energy(),
                         "rel_error_vs_exact": err / nrm}
            s.free()
        ref = np.linalg.norm(fields["f64"])
        for prec in ("f32", "bf16x3"):
            d = fields[prec] - fields["f64"]
            row[f"{prec}_vs_f64_rel_per_field"] = [float(np.linalg.norm(d[f]) / ref) for f in range(6)]
            row[f"{prec}_vs_f64_rel"] = float(np.linalg.norm(d) / ref)
            row[f"energy_drift_{prec}_over_f64"] = row[prec]["energy_T"] / row["f64"]["energy_T"] - 1.0
        results.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    out = {"metric": "precision sweep: FP32 and split-BF16 vs FP64 error, energy drift, error vs exact mode",
           "value": results[0]["f32_vs_f64_rel"], "unit": "relative L2", "n_gpus": 1,
           "higher_is_better": False, "data": "synthetic",
           "config": {"workload": f"(1,1,0) cavity mode, jittered permuted cubes, N=5 on 6*{args.sweep_n5}^3 "
                                  f"tets to t={args.sweep_t} and N=7 on 6*{args.sweep_n7}^3 tets to "
                                  f"t={args.sweep_t7}, FP64, FP32 and split-BF16, same step (CFL 0.5)"},
           "results": results}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--order", type=int, default=4)
    ap.add_argument("--n", type=int, default=40)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=20)
    ap.add_argument("--reps", type=int, default=20,
                    help="repetitions of a two-step graph replay for the per-launch median / p10 / p90")
    ap.add_argument("--batch", action="store_true",
                    help="batched form: 64 meshes of mixed size and order, batched vs plain loop")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--precision-sweep", action="store_true",
                    help="precision form: cavity mode in FP64 and FP32 at N = 5 and 7")
    ap.add_argument("--sweep-t", type=float, default=1.0)
    ap.add_argument("--sweep-n5", type=int, default=32)
    ap.add_argument("--sweep-n7", type=int, default=32)
    ap.add_argument("--sweep-t7", type=float, default=0.1)
    ap.add_argument("--serve", action="store_true",
                    help="serving form: Poisson arrivals of cavity solves, continuous admission vs FIFO")
    ap.add_argument("--serve-requests", type=int, default=24)
    ap.add_argument("--no-solves", action="store_true",
                    help="skip the compact batched and served legs of the default run")
    ap.add_argument("--solves-batch-steps", type=int, default=100)
    ap.add_argument("--solves-serve-requests", type=int, default=12)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--serve-chunk", type=int, default=64)
    ap.add_argument("--serve-backfill", action="store_true",
                    help="oldest request first, then the arrived request of least work")
    ap.add_argument("--material", action="store_true",
                    help="heterogeneous medium (eps, mu log-uniform in [1, 4]) with absorbing z = 1 faces")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (scales FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the library runs one GPU per process; a multi-GPU domain decomposition is not implemented)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.batch:
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.serve:
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.precision_sweep:
        run_precision_sweep(args)
        return
    if args.copy_calibration:
        n = 256 * 1024 * 1024 // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 3}), flush=True)
        return

    import dginputs
    import paper_0901_1024_amd as P

    N, n, prec = args.order, args.n, args.precision
    Np, Nfp = counts(N)
    word = 8 if prec == "f64" else 4
    t_setup = time.perf_counter()
    v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
    kw = {}
    if args.material:
        eps, mu = dginputs.random_materials(e.shape[0])
        kw = dict(eps=eps, mu=mu, face_bc=dginputs.faces_on_plane(v, e, 2, 1.0) * 2)
    s = P.Solver(v, e, N, prec, reorder=1, device=0, **kw)
    x = s.nodes()
    u0 = dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x[0], x[1], x[2])
    del x
    s.set_fields(u0)
    dt = s.stable_dt(0.5)
    K = s.K
    t_setup = time.perf_counter() - t_setup
    print(f"setup done: K={K} N={N} {prec} dt={dt:.4e} ({t_setup:.1f} s)", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    e0 = s.energy()
    s.solve(dt, args.warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record(stream)
    s.solve(dt, args.steps)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = start.elapsed_time(stop)
    # per-launch spread: repetitions of a two-step (ten-launch) graph replay, each between
    # HIP events on the same stream
    reps = []
    for _ in range(args.reps):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.solve(dt, 2)
        z.record(stream)
        z.synchronize()
        reps.append(a.elapsed_time(z) * 1e3 / 10.0)
    reps_us = np.array(reps)
    # the exported right-hand side (dg_rhs: canonical arrays in and out, two permutes around
    # one stage kernel in right-hand-side mode), median of 10 calls
    u_c = torch.empty(6 * K * Np, dtype=torch.float64 if prec == "f64" else torch.float32, device="cuda")
    s.get_fields(out=u_c)
    r_c = torch.empty_like(u_c)
    rhs_us = []
    for _ in range(10):
        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        s.rhs(u_c, r_c)
        z.record(stream)
        z.synchronize()
        rhs_us.append(a.elapsed_time(z) * 1e3)
    del u_c, r_c
    e1 = s.energy()
    print(f"timed {args.steps} steps: {ms:.3f} ms (wall {wall * 1e3:.1f} ms); energy {e0:.6e} -> {e1:.6e}",
          file=sys.stderr, flush=True)
    if not (e1 <= e0 * (1 + 1e-5)):
        print("energy grew: result invalid", file=sys.stderr)
        sys.exit(1)

    launches = 5 * args.steps
    sec = ms / 1e3
    per_launch_s = sec / launches
    flops_launch = K * flops_per_elem_stage(N)
    bytes_launch = K * bytes_per_elem_stage(N, word, args.material)
    gflops = flops_launch * launches / sec / 1e9
    gbs = bytes_launch / per_launch_s / 1e9
    tflops_k = flops_launch / per_launch_s / 1e12
    t_hbm = bytes_launch / (HBM_PEAK_GBS * 1e9)
    t_cmp = flops_launch / (PEAKS_TFLOPS[prec] * 1e12)
    if t_hbm >= t_cmp:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        roof = {"bound": "mfma", "achieved": round(tflops_k, 2), "peak": PEAKS_TFLOPS[prec], "unit": "TFLOP/s",
                "frac": round(tflops_k / PEAKS_TFLOPS[prec], 4)}
    roof["traffic"] = None if args.material else recorded_traffic(N, prec, K)
    mat = "true" if args.material else "false"
    roof["kernel"] = (f"smfma_stage_kernel<{N},true,{mat},false>" if prec == "f32" and N == 3
                      else f"mfma_stage_kernel<{N},true,{mat},false>" if prec == "f32" and N == 4
                      else f"hmfma_stage_kernel<{N},true,{mat},false>" if prec == "f32" and N in (5, 6, 7)
                      else f"dmfma_stage_kernel<{N},true,{mat},false>" if prec == "f64" and N == 3
                      else f"wmfma_stage_kernel<{N},true,{mat},false>" if prec == "f64" and N in (4, 5, 6, 7)
                      else f"bmfma_stage_kernel<{N},true,{mat},false>" if prec == "bf16x3"
                      else f"stage_kernel<{'float' if prec == 'f32' else 'double'},{N},true>")
    roof["hbm_gbs_algorithmic"] = round(gbs, 1)
    roof["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    roof["tflops_algorithmic"] = round(tflops_k, 2)
    roof["us_per_launch"] = round(per_launch_s * 1e6, 2)
    roof["dg_rhs_us"] = round(float(np.median(rhs_us)), 2)
    # attainable HBM bandwidth on this GPU: a plain 1 GiB device-to-device copy (read + write),
    # median of 10, beside the nominal 8 TB/s
    copy_gbs = device_copy_gbs(torch)
    roof["copy_gbs_measured"] = round(copy_gbs, 1)
    roof["hbm_frac_of_copy"] = round(gbs / copy_gbs, 4)
    if len(reps_us):
        roof["launch_us_reps"] = {"median": round(float(np.median(reps_us)), 2),
                                  "p10": round(float(np.percentile(reps_us, 10)), 2),
                                  "p90": round(float(np.percentile(reps_us, 90)), 2), "reps": len(reps_us),
                                  "launches_per_rep": 10}

    out = {
        "metric": METRIC,
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": f"nodal DG Maxwell LSRK4, unit cube 6*{n}^3={K} jittered+permuted tets, "
                               f"N={N}, {prec}, "
                               + ("random eps/mu in [1,4], absorbing z=1 faces, other walls PEC"
                                  if args.material else "vacuum, PEC walls")
                               + ", random smooth fields",
                   "order": N, "K": K, "Np": Np, "stages_per_step": 5, "parallelism": "single GPU"},
        "hbm_gbs": round(gbs, 1),
        "dof_rhs_per_s": round(6 * Np * K * launches / sec, 1),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(N, args.cpu_sample_n)
        cb["speedup_gpu_over_oracle"] = round(gflops / cb["value"], 1)
        cb["speedup_gpu_over_one_core"] = round(gflops / cb["one_core"]["value"], 1)
        out["cpu_baseline"] = cb
    if not args.no_solves:
        # the metric's second half, compact: solves/s of the batched form against the plain
        # per-mesh loop, and solves/s + p50/p99 latency of continuous admission against the
        # plain FIFO loop at the FIFO capacity rate (smaller runs than --batch / --serve)
        s.free()
        args.batch_steps = args.solves_batch_steps
        bt = run_batch(args)
        args.serve_requests = args.solves_serve_requests
        sv = run_serve(args, rates=(1.0,))
        row = sv["sweep"][0]
        out["solves"] = {
            "batched": {"workload": bt["config"]["workload"], "solves_per_s": bt["value"],
                        "plain_solves_per_s": bt["plain_solves_per_s"],
                        "speedup_over_plain": bt["speedup_batched_over_plain"]},
            "served": {"workload": sv["config"]["workload"] + " at the FIFO capacity rate",
                       "slots": args.serve_slots, "solves_per_s": row["served"]["solves_per_s"],
                       "p50_s": row["served"]["p50_latency_s"], "p99_s": row["served"]["p99_latency_s"],
                       "fifo_solves_per_s": row["fifo"]["solves_per_s"], "fifo_p50_s": row["fifo"]["p50_latency_s"],
                       "fifo_p99_s": row["fifo"]["p99_latency_s"]},
        }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Autotuner for the stage kernel choice (dg_opts.tile_id).

The paper generates and searches kernel variants per order and problem size (Sec. 1, the
generative approach; Sec. 6, the method-parameter table). Here the search space is the kernel
family of each order and precision: the element-wise kernel (one thread per element node, as
many workgroups as tiles of 256 / Np elements) against the contraction kernel (16- or
8-element tiles on the matrix cores, a persistent grid), which differ most on small meshes
that do not fill the device, and at FP32 N = 3 also the tile shape of the contraction kernel
(8 or 16 elements). tune() times the candidates on synthetic meshes of each size bucket
(jittered, permuted Kuhn cubes, smooth fields; a number of graph-replayed steps after a warm-up)
and stores the fastest per (precision, order, size) in a JSON table; choose() reads the table
(the nearest bucket in log size) for Solver(..., tile_id="auto").
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULT_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning.json")
_cache = {}


def _path():
    return os.environ.get("DG_TUNING_FILE", DEFAULT_PATH)


def load(path=None):
    path = path or _path()
    if path not in _cache:
        try:
            with open(path) as fh:
                _cache[path] = json.load(fh)
        except (OSError, ValueError):
            _cache[path] = {}
    return _cache[path]


def choose(order, precision, K, path=None):
    """tile_id for this order, precision and mesh size: the table's choice at the nearest size
    bucket (log scale), or 0 (the library's default) without an entry."""
    rows = load(path).get("choices", {}).get(f"{precision}/{order}")
    if not rows:
        return 0
    best = min(rows, key=lambda r: abs(math.log(max(K, 1)) - math.log(r["K"])))
    return int(best["tile_id"])


def candidates(order, precision):
    """Kernel families available for this order and precision (tile_id values)."""
    if precision == "bf16x3":
        return [2] if 5 <= order <= 7 else []
    out = []
    if not (precision == "f32" and order == 4):      # FP32 N = 4 rows are padded for the matrix cores
        out.append(1)
    if (precision == "f32" and 3 <= order <= 7) or (precision == "f64" and 3 <= order <= 7):
        out.append(2)
    if precision == "f32" and order == 3:            # 16-element contraction tiles
        out.append(3)
    return out


def tune(orders=range(1, 10), precisions=("f32", "f64"), sizes=(750, 6000, 48000, 384000), steps=20,
         path=None, device=0, log=print):
    """Time every candidate kernel per (precision, order, size) and write the table."""
    import numpy as np
    import torch

    import dginputs
    from . import Solver

    table = {"what": "faster stage kernel (tile_id) per precision/order and mesh size; "
                     f"{steps} graph-replayed RK steps after 4 warm-up steps, median of 3",
             "device": torch.cuda.get_device_name(device), "choices": {}, "timings": {}}
    for prec in precisions:
        for N in orders:
            cand = candidates(N, prec)
            if not cand:
                continue
            rows, times = [], []
            for size in sizes:
                n = max(1, round((size / 6.0) ** (1.0 / 3.0)))
                v, e = dginputs.kuhn_cube(n, jitter=0.15, permute=True)
                per = {}
                for tid in cand:
                    s = Solver(v, e, N, prec, device=device, tile_id=tid)
                    x = s.nodes()
                    s.set_fields(dginputs.eval_smooth_fields(dginputs.smooth_field_modes(), x[0], x[1], x[2]).astype(s.dtype))
                    dt = s.stable_dt()
                    s.solve(dt, 4)
                    reps = []
                    for _ in range(3):
                        a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                        a.record()
                        s.solve(dt, steps)
                        z.record()
                        z.synchronize()
                        reps.append(a.elapsed_time(z) * 1e3 / steps)
                    per[tid] = float(np.median(reps))
                    s.free()
                best = min(per, key=per.get)
                rows.append({"K": int(e.shape[0]), "tile_id": int(best)})
                times.append({"K": int(e.shape[0]), "us_per_step": {str(k): round(v, 2) for k, v in per.items()}})
                log(f"tune {prec} N={N} K={e.shape[0]}: " + ", ".join(f"tile {k}: {v:.1f} us" for k, v in per.items()))
            table["choices"][f"{prec}/{N}"] = rows
            table["timings"][f"{prec}/{N}"] = times
    path = path or _path()
    with open(path, "w") as fh:
        json.dump(table, fh, indent=1)
    _cache.pop(path, None)
    return table


if __name__ == "__main__":
    tune()

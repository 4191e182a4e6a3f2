"""Serving form: continuous admission of DG solves on one GPU.

Requests (a mesh, an order, a step count and initial fields) arrive over time. The server
admits a request as soon as a slot is free and its device footprint (dg_setup_query) fits the
memory budget; the host-side setup (mesh build, upload) runs in worker threads, and every
admitted solve advances on its own stream in chunks of steps, so requests that arrive while
others run are taken in and their work overlaps on the device. A finished solve releases its
workspace, which admits the next ones. With one slot the same loop is the plain first-in,
first-out baseline. Each solve's arithmetic is independent of the others, so its result is the
same alone and in the mix.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field
from typing import Any, Callable, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float                    # seconds after the start of the run
    vxyz: np.ndarray
    etov: np.ndarray
    order: int
    steps: int
    init: Callable[[np.ndarray], np.ndarray]   # node coordinates (3, K, Np) -> fields (6, K, Np)
    precision: str = "f32"
    cfl: float = 0.5
    face_bc: Optional[np.ndarray] = None
    eps: Optional[np.ndarray] = None
    mu: Optional[np.ndarray] = None
    deadline: Optional[float] = None  # seconds after arrival; a solve not done by then is cancelled
    # filled in by the server
    footprint: int = 0
    t_admit: Optional[float] = None
    t_start: Optional[float] = None
    t_done: Optional[float] = None
    result: Optional[np.ndarray] = None
    error: Optional[str] = None       # set when the numeric monitor stopped the solve or it was cancelled

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class _Active:
    req: Request
    solver: Any
    stream: Any
    dt: float
    left: int
    event: Any = None
    e0: Optional[float] = None        # energy at admission (numeric monitor)


def work(r):
    """Work estimate of a request: steps x elements x Np^2 (the contraction dominates)."""
    Np = (r.order + 1) * (r.order + 2) * (r.order + 3) // 6
    return r.steps * r.etov.shape[0] * Np * Np


def _percentile(v, q):
    return float(np.percentile(np.asarray(v, dtype=np.float64), q)) if len(v) else float("nan")


def summary(done):
    """Throughput and latency of completed requests (requests stopped by the numeric monitor
    are counted apart)."""
    failed = [r for r in done if r.error is not None]
    done = [r for r in done if r.error is None]
    if not done:
        return {"completed": 0, "failed": len(failed)}
    t_end = max(r.t_done for r in done)
    t_first = min(r.arrival for r in done)
    lat = [r.latency for r in done]
    return {"completed": len(done), "makespan_s": t_end - t_first,
            "solves_per_s": len(done) / (t_end - t_first) if t_end > t_first else float("nan"),
            "p50_latency_s": _percentile(lat, 50), "p99_latency_s": _percentile(lat, 99),
            "mean_latency_s": float(np.mean(lat)), "failed": len(failed)}


class Server:
    """budget_bytes: device memory the admitted solves may hold together; slots: solves in
    flight at once (default 4, the hardware queues a process gets: more streams would share
    queues and serialise); backfill: the first free slot takes the oldest waiting request, any
    further one the arrived request of least work (so small solves run beside a large one
    instead of queueing behind it); chunk_steps: steps issued per scheduling round (even, so a solve reuses its
    captured two-step graph); keep_results: copy each final state to the host; checks: after
    every chunk, a solve whose energy is not finite or has grown (more than check_tol relative
    to its energy at admission) is stopped and reported with `error`, and its memory freed; the
    other solves are not affected. cancel(rid), from any thread while run() is going, or a
    request's deadline, stops a request: a waiting one leaves the queue, a running one is
    released once its current chunk has finished; it is reported with `error` and no result."""

    def __init__(self, budget_bytes: int, slots: int = 4, chunk_steps: int = 64, device: int = 0,
                 keep_results: bool = False, setup_threads: int = 4, backend=None, checks: bool = False,
                 check_tol: float = 1e-4, backfill: bool = False):
        if chunk_steps < 2 or chunk_steps % 2:
            raise ValueError("chunk_steps must be even and >= 2")
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.chunk = int(chunk_steps)
        self.device = device
        self.keep = keep_results
        self.setup_threads = setup_threads
        self.backend = backend if backend is not None else _DeviceBackend(device)
        self.checks = checks
        self.check_tol = check_tol
        self.backfill = backfill
        self._cancel_lock = threading.Lock()
        self._cancelled = set()

    def cancel(self, rid):
        """Ask run() to stop request rid (thread-safe; a no-op for finished requests). A
        cancellation holds for the run that is going: when run() returns it forgets the ids of
        the requests it was given, so a later run may reuse them."""
        with self._cancel_lock:
            self._cancelled.add(rid)

    def _stop_wanted(self, r, now):
        if r.deadline is not None and now - r.arrival > r.deadline:
            return f"cancelled: deadline of {r.deadline} s passed"
        with self._cancel_lock:
            if r.rid in self._cancelled:
                return "cancelled"
        return None

    def run(self, requests, clock=time.perf_counter, idle_sleep=2e-4):
        pending = sorted(requests, key=lambda r: r.arrival)
        for r in pending:
            r.footprint = self.backend.footprint(r)
            if r.footprint > self.budget:
                raise ValueError(f"request {r.rid} needs {r.footprint} B, more than the budget")
        used = 0
        setting_up, active, done = [], [], []
        lock = threading.Lock()
        t0 = clock()
        with ThreadPoolExecutor(max_workers=self.setup_threads) as pool:
            while pending or setting_up or active:
                now = clock() - t0
                # cancelled or overdue requests leave the queue before admission
                for r in [r for r in pending if r.arrival <= now]:
                    why = self._stop_wanted(r, now)
                    if why:
                        pending.remove(r)
                        r.error, r.t_done = why, now
                        done.append(r)
                # admit while a slot and memory are free: the oldest waiting request first;
                # with the backfill policy a slot beyond the first goes to the arrived request
                # of least work instead
                while len(setting_up) + len(active) < self.slots:
                    arrived = [r for r in pending if r.arrival <= now]
                    if not arrived:
                        break
                    r = arrived[0]
                    if self.backfill and (setting_up or active):
                        r = min(arrived, key=work)
                    if used + r.footprint > self.budget:
                        break
                    pending.remove(r)
                    used += r.footprint
                    r.t_admit = now
                    setting_up.append((r, pool.submit(self.backend.setup, r)))
                progressed = False
                for item in list(setting_up):
                    r, fut = item
                    if fut.done():
                        solver, stream, dt = fut.result()
                        setting_up.remove(item)
                        r.t_start = clock() - t0
                        active.append(_Active(r, solver, stream, dt, r.steps))
                        progressed = True
                for a in list(active):
                    if a.event is not None and not self.backend.finished(a.event):
                        continue
                    why = self._stop_wanted(a.req, clock() - t0) if a.left > 0 else None
                    if why:   # the stream is idle here: release the solve
                        a.req.error = why
                        a.req.t_done = clock() - t0
                        self.backend.release(a.solver)
                        used -= a.req.footprint
                        active.remove(a)
                        done.append(a.req)
                        progressed = True
                        continue
                    if self.checks:
                        # the stream is idle here (its last chunk has finished)
                        e = self.backend.energy(a.solver, a.stream)
                        if a.e0 is None and np.isfinite(e):
                            a.e0 = e
                        if not np.isfinite(e) or e > a.e0 * (1.0 + self.check_tol):
                            a.req.error = f"numeric monitor: energy {e!r} after {a.req.steps - a.left} steps"
                            a.req.t_done = clock() - t0
                            self.backend.release(a.solver)
                            used -= a.req.footprint
                            active.remove(a)
                            done.append(a.req)
                            progressed = True
                            continue
                    if a.left > 0:
                        n = min(self.chunk, a.left)
                        a.event = self.backend.advance(a.solver, a.stream, a.dt, n)
                        a.left -= n
                        progressed = True
                        continue
                    # all steps issued and the last chunk has finished
                    if self.keep:
                        a.req.result = self.backend.fetch(a.solver, a.stream)
                    a.req.t_done = clock() - t0
                    self.backend.release(a.solver)
                    used -= a.req.footprint
                    active.remove(a)
                    done.append(a.req)
                    progressed = True
                if not progressed:
                    time.sleep(idle_sleep)
        with self._cancel_lock:
            self._cancelled.difference_update(r.rid for r in done)
        return done


class _DeviceBackend:
    """The library on one GPU, one stream per admitted solve (default priority)."""

    def __init__(self, device):
        self.device = device

    def footprint(self, r):
        from . import setup_query
        return setup_query(r.vxyz, r.etov, r.order, r.precision, eps=r.eps, mu=r.mu)

    def setup(self, r):
        import torch
        from . import Solver
        with torch.cuda.device(self.device):
            stream = torch.cuda.Stream(self.device)
            s = Solver(r.vxyz, r.etov, r.order, r.precision, device=self.device, face_bc=r.face_bc,
                       eps=r.eps, mu=r.mu, stream=stream)
            u0 = np.asarray(r.init(s.nodes()))
            s.set_fields(u0.astype(s.dtype), stream=stream)
            stream.synchronize()
            return s, stream, s.stable_dt(r.cfl)

    def advance(self, solver, stream, dt, n):
        import torch
        solver.solve(dt, n, stream=stream)
        ev = torch.cuda.Event()
        ev.record(stream)
        return ev

    def finished(self, event):
        return event.query()

    def energy(self, solver, stream):
        return solver.energy(stream=stream)

    def fetch(self, solver, stream):
        out = solver.get_fields(stream=stream)
        return out

    def release(self, solver):
        solver.free()

"""The serving loop's admission and accounting on the host (a fake device: no GPU)."""
import numpy as np
import pytest

from paper_0901_1024_amd.serve import Request, Server, summary


class FakeBackend:
    """Footprint = 100 B per element; a chunk of n steps takes n polls to finish."""

    def __init__(self):
        self.in_flight = 0
        self.max_in_flight = 0
        self.used = 0
        self.max_used = 0

    def footprint(self, r):
        return 100 * r.etov.shape[0]

    def setup(self, r):
        self.in_flight += 1
        self.used += self.footprint(r)
        self.max_in_flight = max(self.max_in_flight, self.in_flight)
        self.max_used = max(self.max_used, self.used)
        return [r], None, 1.0

    def advance(self, solver, stream, dt, n):
        return {"polls": n}

    def finished(self, ev):
        ev["polls"] -= 1
        return ev["polls"] <= 0

    def fetch(self, solver, stream):
        return np.zeros(1)

    def release(self, solver):
        self.in_flight -= 1
        self.used -= self.footprint(solver[0])


def _requests(Ks, arrivals, steps=6):
    return [Request(rid=i, arrival=a, vxyz=np.zeros((4, 3)), etov=np.zeros((K, 4), dtype=np.int32),
                    order=3, steps=steps, init=lambda x: x)
            for i, (K, a) in enumerate(zip(Ks, arrivals))]


def test_admission_respects_budget_and_slots():
    be = FakeBackend()
    reqs = _requests([10, 20, 30, 40, 50, 60], [0.0] * 6)
    done = Server(budget_bytes=100 * 70, slots=3, chunk_steps=2, backend=be).run(reqs)
    assert len(done) == 6 and be.in_flight == 0
    assert be.max_used <= 100 * 70 and be.max_in_flight <= 3
    assert all(r.t_done >= r.t_admit >= r.arrival for r in done)


def test_one_slot_is_first_in_first_out():
    be = FakeBackend()
    reqs = _requests([5, 5, 5, 5], [0.0, 0.0, 0.0, 0.0])
    done = Server(budget_bytes=10 ** 9, slots=1, chunk_steps=2, backend=be).run(reqs)
    assert [r.rid for r in done] == [0, 1, 2, 3]
    assert be.max_in_flight == 1
    s = summary(done)
    assert s["completed"] == 4 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_oversized_request_is_refused_and_chunks_are_even():
    with pytest.raises(ValueError):
        Server(budget_bytes=100, slots=2, backend=FakeBackend()).run(_requests([10], [0.0]))
    with pytest.raises(ValueError):
        Server(budget_bytes=10 ** 6, chunk_steps=3, backend=FakeBackend())


class MonitoredBackend(FakeBackend):
    """Energies per request: request 1 turns non-finite after its first chunk, request 2 grows."""

    def __init__(self):
        super().__init__()
        self.calls = {}

    def energy(self, solver, stream):
        r = solver[0]
        k = self.calls.get(r.rid, 0)
        self.calls[r.rid] = k + 1
        if r.rid == 1 and k >= 1:
            return float("nan")
        if r.rid == 2:
            return 1.0 + 0.01 * k
        return 1.0 - 1e-6 * k


def test_numeric_monitor_stops_only_the_bad_requests():
    be = MonitoredBackend()
    reqs = _requests([10, 20, 30, 40], [0.0] * 4, steps=8)
    done = Server(budget_bytes=10 ** 6, slots=4, chunk_steps=2, backend=be, checks=True).run(reqs)
    by = {r.rid: r for r in done}
    assert len(done) == 4
    assert by[1].error and "nan" in by[1].error and by[2].error and by[0].error is None and by[3].error is None
    assert be.in_flight == 0 and be.used == 0          # stopped solves released their memory
    s = summary(done)
    assert s["completed"] == 2 and s["failed"] == 2


def test_backfill_admits_oldest_first_then_smallest():
    be = FakeBackend()
    # request 0 arrives first; then a large one (1) and a small one (2)
    reqs = _requests([50, 40, 5], [0.0, 0.0, 0.0], steps=4)
    done = Server(budget_bytes=10 ** 6, slots=2, chunk_steps=2, backend=be, backfill=True).run(reqs)
    by = {r.rid: r for r in done}
    assert by[0].t_admit <= by[2].t_admit <= by[1].t_admit      # oldest, then least work
    plain = Server(budget_bytes=10 ** 6, slots=2, chunk_steps=2, backend=FakeBackend()).run(
        _requests([50, 40, 5], [0.0, 0.0, 0.0], steps=4))
    pb = {r.rid: r for r in plain}
    assert pb[1].t_admit <= pb[2].t_admit                        # arrival order without backfill


def test_cancel_and_deadline_stop_only_their_requests():
    # a counting clock: one unit per reading, so deadlines are deterministic
    ticks = iter(range(10 ** 9))

    def clock():
        return float(next(ticks))

    class CancellingBackend(FakeBackend):
        """Cancels request 1 from inside its first chunk (as another thread would)."""
        server = None

        def advance(self, solver, stream, dt, n):
            if solver[0].rid == 1:
                self.server.cancel(1)
            return super().advance(solver, stream, dt, n)

    be = CancellingBackend()
    reqs = _requests([10, 20, 30, 40], [0.0] * 4, steps=8)
    reqs[2].deadline = 0.0                       # overdue on arrival: never admitted
    reqs[3].deadline = 1e9
    srv = Server(budget_bytes=10 ** 6, slots=2, chunk_steps=2, backend=be)
    be.server = srv
    done = srv.run(reqs, clock=clock)
    by = {r.rid: r for r in done}
    assert len(done) == 4
    assert by[1].error == "cancelled" and by[1].result is None and by[1].t_admit is not None
    assert by[2].error and "deadline" in by[2].error and by[2].t_admit is None
    assert by[0].error is None and by[3].error is None
    assert be.in_flight == 0 and be.used == 0            # the cancelled solve was released
    s = summary(done)
    assert s["completed"] == 2 and s["failed"] == 2


def test_a_cancellation_does_not_outlive_its_run():
    """Ids cancelled during a run (here each one just after its request finished) are
    forgotten when the run returns: a later run on the same server that reuses the ids
    completes every request."""

    class LateCancel(FakeBackend):
        server = None

        def release(self, solver):
            super().release(solver)
            self.server.cancel(solver[0].rid)     # a cancel that arrives after the finish

    be = LateCancel()
    srv = Server(budget_bytes=10 ** 6, slots=2, chunk_steps=2, backend=be)
    be.server = srv
    for _ in range(2):
        done = srv.run(_requests([10, 20, 30], [0.0] * 3))
        assert len(done) == 3 and all(r.error is None for r in done)
    assert be.in_flight == 0 and be.used == 0

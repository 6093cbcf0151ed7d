"""Admission and scheduling policy of the reconstruction service, driven by
a fake executor and a fake clock (no GPU)."""
import numpy as np
import pytest

from paper_2008_11511_amd.serve import Request, Scheduler, make_trace, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def tick(self):
        self.t += 0.01


class FakeExecutor:
    """A request needs `frames` bytes and takes frames/1000 s of device time;
    work of concurrent requests shares the device (processor sharing)."""

    def __init__(self, clock, overlap=True):
        self.clock = clock
        self.overlap = overlap
        self.active = {}
        self.max_used = 0

    def footprint(self, r):
        return r.wl.n_frames

    def start(self, r):
        self.active[r.rid] = [r, r.wl.n_frames / 1000.0, self.clock()]
        return r.rid

    def advance(self, h):
        pass

    def finished(self, h):
        r, need, last = self.active[h]
        now = self.clock()
        share = 1.0 / len(self.active) if not self.overlap else 1.0
        need -= (now - last) * share
        self.active[h] = [r, need, now]
        return need <= 1e-12

    def collect(self, h):
        return {"rid": h}

    def release(self, h):
        self.active.pop(h)


def run(budget, sequential=False, n=20, max_active=8):
    clock = FakeClock()
    ex = FakeExecutor(clock)
    reqs = make_trace(n, rate=10.0, seed=3, max_frames=2000)
    sch = Scheduler(ex, budget, max_active=max_active, sequential=sequential, clock=clock, idle=clock.tick)
    sch.run(reqs)
    return reqs, sch.log


def test_every_request_completes_and_memory_stays_within_budget():
    reqs, log = run(budget=3000)
    assert all(r.done is not None and r.result == {"rid": r.rid} for r in reqs)
    assert max(u for _, _, _, u in log) <= 3000
    assert all(r.admitted >= r.arrival - 1e-9 and r.done >= r.admitted for r in reqs)
    s = summarize(reqs, max(r.done for r in reqs))
    assert s["requests"] == 20 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_sequential_mode_runs_one_at_a_time_in_arrival_order():
    reqs, log = run(budget=10 ** 9, sequential=True)
    admits = [rid for kind, rid, _, _ in log if kind == "admit"]
    assert admits == sorted(admits, key=lambda i: (reqs[i].arrival, i))
    active = 0
    for kind, *_ in log:
        active += 1 if kind == "admit" else -1
        assert active <= 1


def test_continuous_batching_overlaps_requests_and_cuts_latency():
    seq, _ = run(budget=10 ** 9, sequential=True)
    con, log = run(budget=10 ** 9, max_active=8)
    active, peak = 0, 0
    for kind, *_ in log:
        active += 1 if kind == "admit" else -1
        peak = max(peak, active)
    assert peak > 1
    assert np.percentile([r.latency for r in con], 99) < np.percentile([r.latency for r in seq], 99)


def test_backfill_admits_smaller_requests_when_the_head_is_blocked_by_memory():
    clock = FakeClock()
    ex = FakeExecutor(clock)
    from synth import Workload
    def wl(j):
        return Workload("t", 64, 1, j, (256, 256), 6.0, 1e6, 0.0, "dm", (1,), 1)
    reqs = [Request(0, 0.0, wl(900)), Request(1, 0.001, wl(900)), Request(2, 0.002, wl(50)),
            Request(3, 0.003, wl(50))]
    sch = Scheduler(ex, 1000, max_active=8, clock=clock, idle=clock.tick)
    sch.run(reqs)
    admits = [rid for kind, rid, _, _ in sch.log if kind == "admit"]
    assert admits[0] == 0
    assert admits.index(2) < admits.index(1)       # small ones fill the memory left by request 0
    with pytest.raises(ValueError):
        Scheduler(ex, 100, clock=clock, idle=clock.tick).run([Request(9, 0.0, wl(900))])

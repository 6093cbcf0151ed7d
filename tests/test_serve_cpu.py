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

    def advance(self, h, slot=0):
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


def test_arena_first_fit_and_coalescing():
    from paper_2008_11511_amd.serve import Arena
    a = Arena(10 * 4096)
    x = a.alloc(3 * 4096)
    y = a.alloc(1)                 # rounded to one page
    z = a.alloc(4 * 4096)
    assert (x, y, z) == (0, 3 * 4096, 4 * 4096)
    assert a.alloc(3 * 4096) is None and a.largest_hole() == 2 * 4096
    a.release(y, 1)
    a.release(x, 3 * 4096)
    assert a.largest_hole() == 4 * 4096          # x and y merged
    a.release(z, 4 * 4096)
    assert a.free == [(0, 10 * 4096)]


class QuantumExecutor:
    """Work advances only when the scheduler enqueues it: each advance()
    completes one quantum of a request's remaining work."""

    def __init__(self):
        self.left = {}
        self.advanced = []

    def footprint(self, r):
        return 1

    def start(self, r):
        self.left[r.rid] = r.wl.n_frames
        return r.rid

    def remaining(self, h):
        return self.left[h]

    def advance(self, h, slot=0):
        assert slot == 0
        self.advanced.append(h)
        self.left[h] = max(0, self.left[h] - 100)

    def finished(self, h):
        return self.left[h] == 0

    def collect(self, h):
        return {}

    def release(self, h):
        self.left.pop(h)


def _burst(order, max_running):
    clock = FakeClock()
    ex = QuantumExecutor()
    reqs = make_trace(12, rate=1e6, seed=4, max_frames=2000)     # all present at once
    sch = Scheduler(ex, 10**9, max_active=12, clock=clock, idle=clock.tick, order=order,
                    max_running=max_running)
    sch.run(reqs)
    done = [e[1] for e in sch.log if e[0] == "done"]
    return reqs, done, ex


def test_srpt_running_set_finishes_shortest_first():
    reqs, done, ex = _burst("srpt", 1)
    frames = {r.rid: r.wl.n_frames for r in reqs}
    # every request admitted in the first pass, so completion is by size
    assert [frames[d] for d in done] == sorted(frames[d] for d in done)


def test_fifo_running_set_serves_in_admission_order():
    reqs, done, ex = _burst("fifo", 1)
    assert done == sorted(done, key=lambda rid: next(r.admitted for r in reqs if r.rid == rid))
    # one request's work at a time: its quanta are contiguous in the advance log
    runs = [k for i, k in enumerate(ex.advanced) if i == 0 or ex.advanced[i - 1] != k]
    assert len(runs) == len(set(runs)) == len(reqs)


def test_order_argument_checked():
    with pytest.raises(ValueError):
        Scheduler(QuantumExecutor(), 1, order="lifo")


class WorkingExecutor(QuantumExecutor):
    """Each advance() is one quantum of device time on the fake clock."""

    def __init__(self, clock):
        super().__init__()
        self.clock = clock

    def advance(self, h, slot=0):
        super().advance(h, slot)
        self.clock.t += 0.01


def test_age_cap_puts_an_old_request_ahead_of_shorter_ones():
    # a long request (20 quanta) arrives first; short ones (2 quanta) keep
    # arriving at 80% load.  Pure SRPT lets every short one pass; with an age
    # cap the long one runs to the end once it is older than the cap.
    long_wl = make_trace(1, rate=1.0, seed=2, max_frames=2000, min_frames=2000)[0].wl
    short_wl = make_trace(1, rate=1.0, seed=3, max_frames=200, min_frames=200)[0].wl

    def run(age_cap):
        clock = FakeClock()
        reqs = [Request(0, 0.0, long_wl)] + [Request(i, 0.025 * i, short_wl) for i in range(1, 60)]
        sch = Scheduler(WorkingExecutor(clock), 10**9, max_active=64, clock=clock, idle=clock.tick,
                        order="srpt", max_running=1, age_cap=age_cap)
        sch.run(reqs)
        return {r.rid: r.done - r.arrival for r in reqs}

    srpt, capped = run(None), run(0.3)
    # 0.2 s of work: about 0.3 s of waiting at most, then it runs alone
    assert capped[0] < 0.8 < srpt[0]
    # the short ones still go first until the cap is reached
    assert capped[1] < 0.1


class FailingExecutor(QuantumExecutor):
    def start(self, r):
        if r.rid == 3:
            raise ValueError("bad request")
        return super().start(r)


def test_loop_reports_each_request_once_and_isolates_a_failing_start():
    clock = FakeClock()
    ex = FailingExecutor()
    reqs = make_trace(8, rate=50.0, seed=6, max_frames=800)
    pending = sorted(reqs, key=lambda r: r.arrival)
    done = []

    def poll(now):
        out = []
        while pending and pending[0].arrival <= now:
            out.append(pending.pop(0))
        return out

    sch = Scheduler(ex, 10**9, max_active=4, clock=clock, idle=clock.tick, order="srpt", max_running=1)
    sch.loop(poll, lambda: bool(pending), done.append)
    assert sorted(r.rid for r in done) == list(range(8))
    bad = [r for r in done if r.error is not None]
    assert [r.rid for r in bad] == [3] and isinstance(bad[0].error, ValueError)
    assert all(r.result is not None for r in done if r.rid != 3)
    assert not ex.left                                    # every started request was released


def test_near_field_requests_reserve_the_transfer_function_table():
    """The footprint of a near-field scan includes the plan's 2N-entry
    transfer-function table (workspace sizes come from the library, no GPU)."""
    from paper_2008_11511_amd.serve import GpuExecutor, Request, Scan, near_field_of
    import synth
    far = Request(0, 0.0, Scan(64, 2, 50, (160, 160)), (("dm", 2),), data={})
    near = Request(1, 0.0, Scan(64, 2, 50, (160, 160), near_field=0.05), (("dm", 2),), data={})
    ws = {r.rid: dict(GpuExecutor._layout(r))["ws"] for r in (far, near)}
    assert ws[1] >= ws[0] + 2 * 64 * 8
    assert near_field_of(near.wl) == 0.05 and near_field_of(far.wl) is None
    assert near_field_of(synth.workload("nf1024")) == synth.workload("nf1024").fresnel
    assert near_field_of(synth.workload("dm256")) is None


class LaneExecutor(QuantumExecutor):
    """Records which request each running slot advances."""

    def __init__(self):
        super().__init__()
        self.slots = []

    def advance(self, h, slot=0):
        self.slots.append((slot, h))
        self.advanced.append(h)
        self.left[h] = max(0, self.left[h] - 100)


def test_lanes_run_the_oldest_request_beside_the_shortest_others():
    clock = FakeClock()
    ex = LaneExecutor()
    long_wl = make_trace(1, rate=1.0, seed=2, max_frames=2000, min_frames=2000)[0].wl
    short_wl = make_trace(1, rate=1.0, seed=3, max_frames=200, min_frames=200)[0].wl
    reqs = [Request(0, 0.0, long_wl)] + [Request(i, 0.0, short_wl) for i in range(1, 4)]
    sch = Scheduler(ex, 10**9, max_active=8, clock=clock, idle=clock.tick, order="lanes", max_running=2)
    sch.run(reqs)
    # the oldest request holds lane 0 from the first pass on; the short ones
    # take lane 1 one after the other while it runs
    assert ex.slots[0] == (0, 0)
    lane0 = [h for s, h in ex.slots if s == 0]
    lane1 = [h for s, h in ex.slots if s == 1]
    assert set(lane1) == {1, 2, 3}
    first_long_done = sch.log.index(next(e for e in sch.log if e[0] == "done" and e[1] == 0))
    assert all(e[1] != 0 for e in sch.log[:first_long_done] if e[0] == "done") and \
        sum(1 for e in sch.log[:first_long_done] if e[0] == "done") == 3   # the short ones finished beside it
    assert lane0[:5] == [0] * 5

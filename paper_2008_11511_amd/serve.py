"""On-line reconstruction service: continuous batching of ptychography
requests on one GPU.

The paper's command-line scripts serve on-line analysis at the beamline
(Section 5); here a request is one reconstruction (its scan, data and an
algorithm schedule such as 30 DM + 20 ML cycles).  The loop

* admits arriving requests while their HBM footprint fits the budget and a
  slot is free (FIFO, with a bounded backfill of smaller requests when the
  head of the queue is blocked by memory only);
* keeps every admitted reconstruction's state resident on the device, each
  on its own stream, so that the kernels of different requests overlap;
* enqueues cycles in chunks and detects progress and completion with events
  (no blocking synchronisation of the loop);
* frees a request's memory as soon as its result is back on the host, which
  admits the next ones.

Every reconstruction runs with its own plan and its own fixed-order
reductions, so its result does not depend on what else is running.

The policy (`Scheduler`) is separate from the device work (`GpuExecutor`) so
that admission and ordering can be tested with a fake executor and clock.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional

import numpy as np

SCHEDULE = (("dm", 30), ("ml", 20))


@dataclasses.dataclass
class Scan:
    """Sizes of a caller-supplied reconstruction (the fields the service needs)."""
    n: int
    n_modes: int
    n_frames: int
    obj_shape: tuple
    near_field: object = None        # Fresnel parameter(s) of a near-field scan, None = far field


def near_field_of(wl):
    """The near-field Fresnel parameter(s) of a request's scan, or None."""
    if isinstance(wl, Scan):
        return wl.near_field
    return wl.fresnel if getattr(wl, "geometry", "far") == "near" else None


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float                   # seconds after the start of the loop
    wl: object                       # synth.Workload (synthetic data) or Scan
    schedule: tuple = SCHEDULE
    data: Optional[dict] = None      # caller data: iobs, offsets, mask, obj0, probe0
    # filled by the scheduler
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None
    error: Optional[BaseException] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def frame_cycles(self) -> int:
        return self.wl.n_frames * sum(n for _, n in self.schedule)


class Scheduler:
    """Admission and progress policy over an executor.

    executor.footprint(req) -> bytes;  executor.start(req) -> handle;
    executor.advance(handle, slot) -> None (enqueue more work, in running
    slot `slot`, if the pipeline has room);  executor.finished(handle) -> bool;  executor.collect(handle) ->
    result (host);  executor.release(handle).
    """

    def __init__(self, executor, hbm_budget: int, max_active: int = 8, max_backfill: int = 8,
                 sequential: bool = False, clock: Callable[[], float] = time.perf_counter,
                 idle: Callable[[], None] = lambda: time.sleep(2e-4), max_running: Optional[int] = None,
                 order: str = "fifo", age_cap: Optional[float] = None):
        if order not in ("fifo", "srpt", "lanes"):
            raise ValueError("order must be 'fifo', 'srpt' or 'lanes'")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = 1 if sequential else int(max_active)
        self.max_backfill = 0 if sequential else int(max_backfill)
        # of the admitted requests, at most max_running get new work enqueued
        # at a time (the others hold their data resident and wait), chosen
        # by admission order or by least remaining work; with age_cap, a
        # request that arrived more than age_cap seconds ago goes before all
        # younger ones (oldest first), which bounds how long short requests
        # can hold back a long one.  "lanes": the oldest request always runs
        # (in the order of sequential solves), and the other running slots
        # take the least remaining work among the rest, so short requests
        # overlap the long one on the device instead of waiting for it
        self.max_running = self.max_active if max_running is None else max(1, int(max_running))
        self.order = order
        self.age_cap = age_cap
        self.clock = clock
        self.idle = idle
        self.log: List[tuple] = []

    def run(self, requests: List[Request]) -> List[Request]:
        """Serve a trace: each request is submitted at its arrival time."""
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            self.check(r)

        def poll(now):
            out = []
            while pending and pending[0].arrival <= now:
                out.append(pending.pop(0))
            return out

        self.loop(poll, lambda: bool(pending))
        return requests

    def check(self, r: Request) -> None:
        if self.ex.footprint(r) > self.budget:
            raise ValueError(f"request {r.rid} needs {self.ex.footprint(r)} bytes, more than the budget "
                             f"{self.budget}")

    def loop(self, poll: Callable[[float], List[Request]], more: Callable[[], bool],
             on_done: Optional[Callable[[Request], None]] = None) -> None:
        """Run until `more()` is false and every request is done.  poll(now)
        returns the requests that arrived since the last call (arrival times
        on the loop's clock, seconds since `self.t0`)."""
        queue: List[Request] = []
        active = []                  # (req, handle, bytes)
        used = 0
        t0 = self.t0 = self.clock()
        skips = 0
        while True:
            now = self.clock() - t0
            queue.extend(poll(now))
            if not (queue or active or more()):
                break
            # admission: FIFO; when the head is blocked by memory only, later
            # requests that fit may go first, at most max_backfill times
            i = 0
            while i < len(queue) and len(active) < self.max_active:
                r = queue[i]
                need = self.ex.footprint(r)
                if used + need <= self.budget and getattr(self.ex, "fits", lambda q: True)(r):
                    queue.pop(i)
                    r.admitted = self.clock() - t0
                    try:
                        h = self.ex.start(r)
                    except Exception as e:          # this request fails, the others go on
                        r.error = e
                        r.done = self.clock() - t0
                        self.log.append(("error", r.rid, r.done, used))
                        if on_done is not None:
                            on_done(r)
                        continue
                    active.append((r, h, need))
                    used += need
                    self.log.append(("admit", r.rid, r.admitted, used))
                    if i > 0:
                        skips += 1
                    else:
                        skips = 0
                    continue
                if i == 0 and skips >= self.max_backfill:
                    break
                if i >= 0 and self.max_backfill == 0:
                    break
                i += 1
            progressed = False
            for entry in list(active):
                r, h, need = entry
                if self.ex.finished(h):
                    try:
                        r.result = self.ex.collect(h)
                    except Exception as e:        # the request failed on the device
                        r.error = e
                    r.done = self.clock() - t0
                    self.ex.release(h)
                    active.remove(entry)
                    used -= need
                    self.log.append(("done", r.rid, r.done, used))
                    progressed = True
                    if on_done is not None:
                        on_done(r)
            running = list(active)
            if self.order == "srpt":
                now = self.clock() - t0
                cap = math.inf if self.age_cap is None else self.age_cap

                def key(e):
                    r, h, _ = e
                    if now - r.arrival > cap:
                        return (0, r.arrival, r.rid)
                    return (1, self.ex.remaining(h), r.admitted, r.rid)
                running.sort(key=key)
            elif self.order == "lanes" and running:
                oldest = min(running, key=lambda e: (e[0].arrival, e[0].rid))
                rest = sorted((e for e in running if e is not oldest),
                              key=lambda e: (self.ex.remaining(e[1]), e[0].admitted, e[0].rid))
                running = [oldest] + rest
            for slot, (r, h, need) in enumerate(running[:self.max_running]):
                self.ex.advance(h, slot)
            if not progressed:
                self.idle()


def summarize(reqs: List[Request], wall: float) -> dict:
    lat = np.array([r.latency for r in reqs])
    fc = sum(r.frame_cycles for r in reqs)
    return {"requests": len(reqs), "wall_s": round(wall, 3),
            "throughput_req_s": round(len(reqs) / wall, 3),
            "frames_cycles_per_s": round(fc / wall, 1),
            "p50_latency_s": round(float(np.percentile(lat, 50)), 3),
            "p99_latency_s": round(float(np.percentile(lat, 99)), 3),
            "mean_latency_s": round(float(lat.mean()), 3)}


# --------------------------------------------------------------------------
# Device arena
# --------------------------------------------------------------------------

class Arena:
    """First-fit allocator over one contiguous range of `size` bytes, with
    coalescing of free neighbours (offsets only; no device calls)."""

    ALIGN = 4096

    def __init__(self, size: int):
        self.size = int(size)
        self.free = [(0, self.size)]          # sorted (offset, length)

    def alloc(self, n: int) -> Optional[int]:
        n = -(-int(n) // self.ALIGN) * self.ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                return off
        return None

    def release(self, off: int, n: int) -> None:
        n = -(-int(n) // self.ALIGN) * self.ALIGN
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def largest_hole(self) -> int:
        return max((ln for _, ln in self.free), default=0)


# --------------------------------------------------------------------------
# GPU executor
# --------------------------------------------------------------------------

class _Job:
    """Device state of one active request."""


class GpuExecutor:
    """Runs requests with the HIP library on a fixed set of streams.

    Inputs of a request (truth, positions, mask, starts) are prepared on the
    host beforehand by `prepare`; at admission its data are generated on the
    device (library forward model + Poisson draw), which stands in for the
    detector stream arriving.

    Streams: one for admissions (uploads, data, plan tables) and one per
    running slot.  The device has a few hardware queues and streams beyond
    them share one, so a stream per request would let an admission wait
    behind the cycles already queued by a running request; with a fixed set,
    admissions overlap the running work.  A request that moves to another
    slot's stream is ordered after its own last enqueued work by an event.
    """

    def __init__(self, device="cuda:0", chunk: int = 5, depth: int = 2):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.chunk = int(chunk)
        self.depth = int(depth)
        self.host = {}
        self.setup_stream = torch.cuda.Stream(device=self.dev)
        self.run_streams = []
        # the most requests seen with chunks enqueued and not yet complete
        # on the device at the same time (queried from their events)
        self.max_in_flight = 0
        self.jobs = {}

    # -- host preparation (outside the timed trace) -----------------------
    def prepare(self, req: Request) -> None:
        import synth
        from .plan import offsets_from_positions
        wl = req.wl
        near = near_field_of(wl) is not None
        obj = synth.object_truth(wl.obj_shape, wl.seed)
        if near:
            probe = synth.near_field_probe(wl.n, wl.n_modes, wl.seed)
            pos = synth.random_positions(wl.n_frames, wl.step, wl.seed)
        else:
            probe = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
            pos = synth.spiral_positions(wl.n_frames, wl.step)
        offs = offsets_from_positions(pos, wl.n, wl.obj_shape)
        probe = probe * synth.probe_photon_scale(obj, probe, offs, wl.photons)
        mask = synth.gap_mask(wl.n, wl.mask_frac, wl.seed, fft_order=not near)
        self.host[req.rid] = dict(
            obj=np.ascontiguousarray(obj.astype(np.complex64)),
            probe=np.ascontiguousarray(probe.astype(np.complex64)),
            offs=offs, mask=mask,
            obj0=np.ascontiguousarray(synth.start_object(wl.obj_shape).astype(np.complex64)),
            probe0=np.ascontiguousarray(synth.start_probe(probe).astype(np.complex64)))

    def close(self) -> None:
        """Give the arena back to the device."""
        self.pool = None
        self.arena = None
        self.torch.cuda.empty_cache()

    def attach_arena(self, nbytes: int) -> None:
        """Reserve the device memory the service admits requests into."""
        torch = self.torch
        self.pool = torch.empty(int(nbytes), dtype=torch.uint8, device=self.dev)
        self.arena = Arena(int(nbytes))

    @staticmethod
    def _layout(req: Request):
        """Byte layout of one request's contiguous device region."""
        import ctypes
        from ._lib import Desc, check, lib
        wl = req.wl
        n2 = wl.n * wl.n
        no = wl.obj_shape[0] * wl.obj_shape[1]
        from ._lib import FLAG_NEAR_FIELD
        flags = FLAG_NEAR_FIELD if near_field_of(wl) is not None else 0
        d = Desc(wl.n, wl.n_modes, wl.n_frames, wl.obj_shape[0], wl.obj_shape[1], 0, 1e-2, 1e-2, 1e-20, flags)
        ws = ctypes.c_size_t()
        check(lib().ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(ws)))
        synthetic = req.data is None
        n_ml = sum(c for kind, c in req.schedule if kind == "ml")
        parts = [("iobs", 4 * wl.n_frames * n2), ("psi", 8 * wl.n_frames * wl.n_modes * n2),
                 ("ws", int(ws.value)), ("state", 0), ("obj", 8 * no), ("probe", 8 * wl.n_modes * n2),
                 ("obj_t", 8 * no if synthetic else 0), ("probe_t", 8 * wl.n_modes * n2 if synthetic else 0),
                 ("mask", n2), ("llk", 16), ("hist", 8 * max(n_ml, 1)), ("flag", 4)]
        return parts

    @staticmethod
    def footprint(req: Request) -> int:
        """Device bytes a request holds while active (one contiguous region)."""
        wl = req.wl
        no = wl.obj_shape[0] * wl.obj_shape[1]
        n2k = wl.n_modes * wl.n * wl.n
        # CG state: scalars, direction and gradient, partials, and the kept row
        # transforms of every frame (ptycho_ml_state_bytes), with slack for alignment
        state = 8 * 16 + 2 * 8 * no + 2 * 8 * n2k + 8 * 4 * 256 + 8 * 256 * 6 + 8 * n2k * wl.n_frames
        total = 0
        for name, nb in GpuExecutor._layout(req):
            total += (-(-(state if name == "state" else nb) // 4096)) * 4096
        # plus the Poisson draw's temporary, which goes through torch
        return total + GpuExecutor._temp_bytes(req)

    @staticmethod
    def _temp_bytes(req: Request) -> int:
        wl = req.wl
        return 4 * wl.n_frames * wl.n * wl.n if req.data is None else 0

    def fits(self, req: Request) -> bool:
        arena = getattr(self, "arena", None)
        if arena is None:
            return True
        return arena.largest_hole() >= self.footprint(req) - self._temp_bytes(req)

    # -- device work ------------------------------------------------------
    def start(self, req: Request) -> _Job:
        torch = self.torch
        from .plan import Plan
        t_start = time.perf_counter()
        parts = []

        def mark(label):
            parts.append((label, time.perf_counter()))

        h = self.host[req.rid] if req.data is None else req.data
        wl = req.wl
        j = _Job()
        j.req = req
        j.stream = self.setup_stream
        n, k, jj = wl.n, wl.n_modes, wl.n_frames
        region = None
        if getattr(self, "arena", None) is not None:
            size = self.footprint(req) - self._temp_bytes(req)
            off = self.arena.alloc(size)
            if off is None:
                raise RuntimeError("arena has no room (admission should have prevented this)")
            j.region = (off, size)
            region = self.pool[off:off + size]
        else:
            j.region = None

        cursor = [0]

        def carve(nbytes, dtype, shape):
            if region is None:
                return torch.empty(shape, dtype=dtype, device=self.dev)
            c = cursor[0]
            cursor[0] = c + (-(-nbytes // 4096)) * 4096
            return region[c:c + nbytes].view(dtype).view(shape)

        sizes = dict(self._layout(req))
        mark("alloc")

        def upload(dst, x):
            # device tensors are copied on the request's stream; host arrays go
            # through page-locked staging, so the copy is a DMA on that stream
            # and the host does not wait for it
            if isinstance(x, torch.Tensor) and x.is_cuda:
                dst.copy_(x, non_blocking=True)
                return
            t = x if isinstance(x, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(x))
            dst.copy_(t.pin_memory(), non_blocking=True)

        try:
            self._start_on_stream(req, j, h, carve, sizes, upload, mark)
        except BaseException:
            j.plan = None
            if j.region is not None:
                j.stream.synchronize()
                self.arena.release(*j.region)
            raise
        # page-locked result buffers, allocated before any work is enqueued
        j.out_obj = torch.empty(wl.obj_shape, dtype=torch.complex64, pin_memory=True)
        j.out_probe = torch.empty((k, n, n), dtype=torch.complex64, pin_memory=True)
        j.out_llk = torch.empty(2, dtype=torch.float64, pin_memory=True)
        j.out_hist = torch.empty(j.hist.shape, dtype=torch.float64, pin_memory=True)
        j.flag_host = torch.zeros(1, dtype=torch.int32, pin_memory=True)
        j.failed = None
        mark("pinned")
        j.phase = 0
        j.left = req.schedule[0][1]
        j.ml_done = 0
        j.last = torch.cuda.Event()
        j.last.record(j.stream)
        j.events = []
        j.final = None
        j.fresh_ml = True
        self.jobs[req.rid] = j
        j.setup_s = time.perf_counter() - t_start
        prev, j.setup_parts = t_start, {}
        for label, t in parts:
            j.setup_parts[label] = round(t - prev, 4)
            prev = t
        return j

    def _start_on_stream(self, req, j, h, carve, sizes, upload, mark):
        """Device buffers, data and plan of one request, enqueued on j.stream."""
        torch = self.torch
        from .plan import Plan
        wl = req.wl
        n, k, jj = wl.n, wl.n_modes, wl.n_frames
        with torch.cuda.stream(j.stream):
            j.iobs = carve(sizes["iobs"], torch.float32, (jj, n, n))
            j.psi = carve(sizes["psi"], torch.complex64, (jj, k, n, n))
            ws = carve(sizes["ws"], torch.uint8, (sizes["ws"],))
            j.mask = None
            if h.get("mask") is not None:
                j.mask = carve(sizes["mask"], torch.uint8, (n, n))
                upload(j.mask, h["mask"])
            if req.data is None:
                o_t = carve(sizes["obj_t"], torch.complex64, wl.obj_shape)
                p_t = carve(sizes["probe_t"], torch.complex64, (k, n, n))
                upload(o_t, h["obj"])
                upload(p_t, h["probe"])
                mark("upload_truth")
                # data: the forward model written into the data buffer, then the
                # Poisson draw (the plan reads the buffer only from the first cycle on)
                j.plan = Plan(h["offs"], j.iobs, j.mask, k, wl.obj_shape, workspace=ws,
                              near_field=near_field_of(wl))
                mark("plan")
                j.plan.icalc(o_t, p_t, out=j.iobs)
                mark("icalc")
                gen = torch.Generator(device=self.dev)
                gen.manual_seed(int(wl.seed))
                j.iobs.copy_(torch.poisson(j.iobs.clamp_min_(0), generator=gen))
                mark("poisson")
            else:
                if h.get("ready") is not None:
                    j.stream.wait_event(h["ready"])
                upload(j.iobs, h["iobs"])
                mark("upload_data")
                j.plan = Plan(h["offsets"], j.iobs, j.mask, k, wl.obj_shape, workspace=ws,
                              near_field=near_field_of(wl))
                mark("plan")
            j.obj = carve(sizes["obj"], torch.complex64, wl.obj_shape)
            j.probe = carve(sizes["probe"], torch.complex64, (k, n, n))
            upload(j.obj, h["obj0"])
            upload(j.probe, h["probe0"])
            mark("upload_start")
            j.plan.psi_init(j.obj, j.probe, j.psi)
            j.state = carve(self._state_bytes(j.plan), torch.uint8, (self._state_bytes(j.plan),))
            j.llk_buf = carve(16, torch.float64, (2,))
            j.hist = carve(sizes["hist"], torch.float64, (sizes["hist"] // 8,))
            j.flag = carve(4, torch.int32, (1,))
            mark("psi_init")

    @staticmethod
    def _state_bytes(plan) -> int:
        import ctypes
        from ._lib import check, lib
        nb = ctypes.c_size_t()
        check(lib().ptycho_ml_state_bytes(plan._h, ctypes.byref(nb)))
        return int(nb.value)

    @staticmethod
    def remaining(j: _Job) -> float:
        """Work not yet enqueued, in frame-mode-pixel-cycles."""
        wl = j.req.wl
        cycles = j.left + sum(n for _, n in j.req.schedule[j.phase + 1:]) if j.phase < len(j.req.schedule) else 0
        return float(wl.n_frames) * wl.n_modes * wl.n * wl.n * cycles

    def advance(self, j: _Job, slot: int = 0) -> None:
        torch = self.torch
        n_before = len(j.events)
        j.events = [e for e in j.events if not e.query()]
        if len(j.events) < n_before and j.flag_host[0] != 0 and j.failed is None:
            # a chunk's check found a NaN or inf: stop this request
            j.failed = FloatingPointError(f"request {j.req.rid}: non-finite object or probe")
        if j.failed is not None or len(j.events) >= self.depth or j.phase >= len(j.req.schedule):
            return
        while len(self.run_streams) <= slot:
            self.run_streams.append(torch.cuda.Stream(device=self.dev))
        stream = self.run_streams[slot]
        if j.stream is not stream:
            stream.wait_event(j.last)
            j.stream = stream
        with torch.cuda.stream(j.stream):
            while len(j.events) < self.depth and j.phase < len(j.req.schedule):
                kind, _ = j.req.schedule[j.phase]
                n = min(self.chunk, j.left)
                if kind == "dm":
                    j.plan.dm_cycle(j.obj, j.probe, j.psi, n, 3)
                elif kind == "ap":
                    j.plan.ap_cycle(j.obj, j.probe, n, 3, psi=j.psi)
                else:
                    j.plan.ml_cycle(j.obj, j.probe, j.state, n, 3, reset=j.fresh_ml,
                                    hist=j.hist[j.ml_done:j.ml_done + n])
                    j.ml_done += n
                    j.fresh_ml = False
                j.left -= n
                if j.left == 0:
                    j.phase += 1
                    if j.phase < len(j.req.schedule):
                        j.left = j.req.schedule[j.phase][1]
                # failure detection: the flag comes back with the chunk
                j.plan.check_finite(j.obj, j.probe, out=j.flag)
                j.flag_host.copy_(j.flag, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(j.stream)
                j.events.append(ev)
                j.last = ev
                busy = sum(1 for other in self.jobs.values() if any(not e.query() for e in other.events))
                self.max_in_flight = max(self.max_in_flight, busy)
                if j.phase == len(j.req.schedule):
                    j.llk = j.plan.llk(j.obj, j.probe, out=j.llk_buf)
                    j.out_obj.copy_(j.obj, non_blocking=True)
                    j.out_probe.copy_(j.probe, non_blocking=True)
                    j.out_llk.copy_(j.llk, non_blocking=True)
                    j.out_hist.copy_(j.hist, non_blocking=True)
                    j.final = torch.cuda.Event()
                    j.final.record(j.stream)

    def finished(self, j: _Job) -> bool:
        if j.failed is not None:
            return j.last.query()        # nothing of it left in flight
        return j.final is not None and j.final.query()

    def collect(self, j: _Job) -> dict:
        """Host results: final object and probe, LLK per unmasked pixel after
        the last cycle and after each ML cycle, and set-up timing."""
        if j.failed is not None:
            raise j.failed
        if j.flag_host[0] != 0:
            raise FloatingPointError(f"request {j.req.rid}: non-finite object or probe")
        llk = j.out_llk.numpy()
        hist = j.out_hist.numpy()[:j.ml_done] / llk[1]
        return {"obj": j.out_obj.numpy(), "probe": j.out_probe.numpy(), "llk": float(llk[0] / llk[1]),
                "llk_history": hist, "setup_s": j.setup_s, "setup_parts": j.setup_parts}

    def release(self, j: _Job) -> None:
        self.jobs.pop(j.req.rid, None)
        j.plan.close()
        for name in ("plan", "iobs", "mask", "obj", "probe", "psi", "state", "llk", "llk_buf", "hist"):
            setattr(j, name, None)
        if j.region is not None:
            # the region is reused by work enqueued after this point: every
            # kernel of this request precedes its final (or, failed, last) event
            (j.final if j.final is not None else j.last).synchronize()
            self.arena.release(*j.region)
        self.host.pop(j.req.rid, None)


class ReconstructionService:
    """On-line service: reconstructions submitted from any thread are served
    by one loop thread with the policy above; `submit` returns a future.

        with ReconstructionService() as svc:
            fut = svc.submit(iobs, offsets, obj0, probe0, mask)
            res = fut.result()     # obj, probe, llk, llk_history, timings

    Inputs (numpy arrays or torch tensors, host or device): iobs float32
    [J][N][N] (FFT order in the far field), offsets int32 [J][2] window corners, obj0
    complex64 [Ny][Nx] and probe0 complex64 [K][N][N] starting guesses, mask
    uint8 [N][N] (1 = bad pixel) or None.  near_field: the Fresnel
    parameter f or (f_y, f_x) of a near-field scan (iobs and mask then in
    natural pixel order), None for the far field.  The arrays must not change
    until the future is done.  A request whose offsets leave the object, or
    that needs more memory than the budget, is refused in `submit`.
    """

    # The default age cap lets a request be passed by shorter ones only during
    # its first 1/8 s, and at most three requests are admitted (resident) at
    # once, so that few admissions run beside the request on the device: on
    # the mixed trace this keeps every latency statistic at or below
    # one-at-a-time solving; a longer cap (say 1 s) halves the median latency
    # but lets the largest request finish later.
    def __init__(self, device="cuda:0", hbm_budget: Optional[int] = None, max_active: int = 3,
                 max_running: int = 1, order: str = "srpt", age_cap: Optional[float] = 0.125,
                 chunk: int = 5):
        import itertools
        import queue
        import threading
        import torch
        from ._lib import lib
        lib()
        self.ex = GpuExecutor(device, chunk=chunk)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(torch.device(device))
            hbm_budget = int(0.8 * free)
        self.ex.attach_arena(int(hbm_budget))
        self.sch = Scheduler(self.ex, hbm_budget, max_active=max_active, max_running=max_running, order=order,
                             age_cap=age_cap)
        self._in = queue.SimpleQueue()
        self._empty = queue.Empty
        self._closed = threading.Event()
        self._ids = itertools.count()
        self._futures = {}
        self._lock = threading.Lock()
        self._started = threading.Event()
        self._thread = threading.Thread(target=self._run, name="ptycho-serve", daemon=True)
        self._thread.start()
        self._started.wait()

    def submit(self, iobs, offsets, obj0, probe0, mask=None, schedule=SCHEDULE, near_field=None):
        import ctypes
        from concurrent.futures import Future
        import torch
        from ._lib import Desc, check, lib
        if self._closed.is_set():
            raise RuntimeError("the service is closed")
        offs = np.ascontiguousarray(offsets, dtype=np.int32)
        if iobs.ndim != 3 or iobs.shape[1] != iobs.shape[2]:
            raise ValueError("iobs must be [J][N][N]")
        jj, n = int(iobs.shape[0]), int(iobs.shape[1])
        if offs.shape != (jj, 2):
            raise ValueError("offsets must be [J][2]")
        if probe0.ndim != 3 or tuple(probe0.shape[1:]) != (n, n):
            raise ValueError("probe0 must be [K][N][N]")
        if obj0.ndim != 2:
            raise ValueError("obj0 must be [Ny][Nx]")
        if mask is not None and tuple(mask.shape) != (n, n):
            raise ValueError("mask must be [N][N]")
        for kind, cycles in schedule:
            if kind not in ("ap", "dm", "ml") or int(cycles) <= 0:
                raise ValueError(f"bad schedule entry {(kind, cycles)}")
        if near_field is not None and not np.all(np.isfinite(np.asarray(near_field, dtype=np.float64))):
            raise ValueError("near_field must be finite")
        scan = Scan(n, int(probe0.shape[0]), jj, (int(obj0.shape[0]), int(obj0.shape[1])), near_field)
        # sizes and window bounds checked by the library, without GPU work
        d = Desc(n, scan.n_modes, jj, scan.obj_shape[0], scan.obj_shape[1], 0, 1e-2, 1e-2, 1e-20, 0)
        tb = ctypes.c_size_t()
        check(lib().ptycho_plan_dry_run(ctypes.byref(d), offs.ctypes.data, ctypes.byref(tb)))
        ready = None
        if any(isinstance(x, torch.Tensor) and x.is_cuda for x in (iobs, obj0, probe0, mask)):
            # device inputs: the uploads wait for the caller's stream
            ready = torch.cuda.Event()
            ready.record(torch.cuda.current_stream(self.ex.dev))
        r = Request(next(self._ids), 0.0, scan, tuple((k, int(c)) for k, c in schedule),
                    data=dict(iobs=iobs, offsets=offs, obj0=obj0, probe0=probe0, mask=mask, ready=ready))
        self.sch.check(r)
        fut = Future()
        with self._lock:
            self._futures[r.rid] = fut
        self._in.put((r, time.perf_counter()))
        return fut

    def _run(self):
        def poll(now):
            out = []
            while True:
                try:
                    r, t = self._in.get_nowait()
                except self._empty:
                    return out
                r.arrival = max(0.0, t - self.sch.t0)
                out.append(r)

        def done(r):
            with self._lock:
                fut = self._futures.pop(r.rid)
            if r.error is not None:
                fut.set_exception(r.error)
                return
            res = dict(r.result)
            res["timings"] = {"queued_s": r.admitted - r.arrival, "service_s": r.done - r.admitted,
                              "latency_s": r.done - r.arrival, "setup_s": res.pop("setup_s")}
            res.pop("setup_parts", None)
            fut.set_result(res)

        self.sch.t0 = time.perf_counter()
        self._started.set()
        err = None
        try:
            self.sch.loop(poll, lambda: not self._closed.is_set(), done)
        except BaseException as e:             # the loop itself failed: fail what is left
            err = e
        self._closed.set()
        with self._lock:
            left, self._futures = self._futures, {}
        for fut in left.values():
            fut.set_exception(err if err is not None else RuntimeError("the service closed first"))

    def close(self) -> None:
        """Finish the submitted requests, stop the loop and free the arena."""
        self._closed.set()
        self._thread.join()
        self.ex.close()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def make_trace(n_requests: int, rate: float, seed: int = 0, max_frames: int = 2000, sizes=(128, 256, 512),
               schedule=SCHEDULE, min_frames: int = 200, min_side: int = 1024) -> List[Request]:
    import synth
    reqs = []
    for i, (t, wl) in enumerate(synth.serve_requests(n_requests, rate, seed, sizes=sizes,
                                                       frames=(min_frames, max_frames), min_side=min_side)):
        reqs.append(Request(i, t, wl, schedule))
    return reqs


def serve_trace(n_requests: int = 64, rate: float = 2.0, seed: int = 0, hbm_budget: Optional[int] = None,
                max_active: int = 3, sequential: bool = False, device="cuda:0", max_frames: int = 2000,
                sizes=(128, 256, 512), schedule=SCHEDULE, min_frames: int = 200, min_side: int = 1024,
                max_running: Optional[int] = 1, order: str = "srpt", age_cap: Optional[float] = 0.125):
    """Run an arrival trace through the service; returns (requests, summary)."""
    import torch
    reqs = make_trace(n_requests, rate, seed, max_frames, sizes, schedule, min_frames, min_side)
    ex = GpuExecutor(device)
    for r in reqs:
        ex.prepare(r)
    if hbm_budget is None:
        free, total = torch.cuda.mem_get_info(torch.device(device))
        hbm_budget = int(0.8 * free)
    # the arena holds the requests' persistent buffers; the per-request
    # Poisson temporary (counted in the footprint) stays with torch
    ex.attach_arena(int(hbm_budget * 0.85))
    sch = Scheduler(ex, hbm_budget, max_active=max_active, sequential=sequential, max_running=max_running,
                    order=order, age_cap=age_cap)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sch.run(reqs)
    wall = time.perf_counter() - t0
    s = summarize(reqs, wall)
    s["mode"] = "sequential" if sequential else "continuous"
    s["max_active"], s["max_running"], s["order"] = sch.max_active, sch.max_running, sch.order
    s["age_cap_s"] = sch.age_cap
    s["hbm_budget_GB"] = round(hbm_budget / 1e9, 1)
    s["max_requests_in_flight"] = ex.max_in_flight
    ex.close()
    return reqs, s

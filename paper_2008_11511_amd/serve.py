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
class Request:
    rid: int
    arrival: float                   # seconds after the start of the trace
    wl: object                       # synth.Workload
    schedule: tuple = SCHEDULE
    # filled by the scheduler
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def frame_cycles(self) -> int:
        return self.wl.n_frames * sum(n for _, n in self.schedule)


class Scheduler:
    """Admission and progress policy over an executor.

    executor.footprint(req) -> bytes;  executor.start(req) -> handle;
    executor.advance(handle) -> None (enqueue more work if the pipeline has
    room);  executor.finished(handle) -> bool;  executor.collect(handle) ->
    result (host);  executor.release(handle).
    """

    def __init__(self, executor, hbm_budget: int, max_active: int = 8, max_backfill: int = 8,
                 sequential: bool = False, clock: Callable[[], float] = time.perf_counter,
                 idle: Callable[[], None] = lambda: time.sleep(2e-4)):
        self.ex = executor
        self.budget = int(hbm_budget)
        self.max_active = 1 if sequential else int(max_active)
        self.max_backfill = 0 if sequential else int(max_backfill)
        self.clock = clock
        self.idle = idle
        self.log: List[tuple] = []

    def run(self, requests: List[Request]) -> List[Request]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if self.ex.footprint(r) > self.budget:
                raise ValueError(f"request {r.rid} needs {self.ex.footprint(r)} bytes, more than the budget "
                                 f"{self.budget}")
        queue: List[Request] = []
        active = []                  # (req, handle, bytes)
        used = 0
        t0 = self.clock()
        skips = 0
        while pending or queue or active:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.pop(0))
            # admission: FIFO; when the head is blocked by memory only, later
            # requests that fit may go first, at most max_backfill times
            i = 0
            while i < len(queue) and len(active) < self.max_active:
                r = queue[i]
                need = self.ex.footprint(r)
                if used + need <= self.budget:
                    queue.pop(i)
                    r.admitted = self.clock() - t0
                    h = self.ex.start(r)
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
                    r.result = self.ex.collect(h)
                    r.done = self.clock() - t0
                    self.ex.release(h)
                    active.remove(entry)
                    used -= need
                    self.log.append(("done", r.rid, r.done, used))
                    progressed = True
                else:
                    self.ex.advance(h)
            if not progressed:
                self.idle()
        return requests


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
# GPU executor
# --------------------------------------------------------------------------

class _Job:
    """Device state of one active request."""


class GpuExecutor:
    """Runs requests with the HIP library, one stream per active request.

    Inputs of a request (truth, positions, mask, starts) are prepared on the
    host beforehand by `prepare`; at admission its data are generated on the
    device (library forward model + Poisson draw), which stands in for the
    detector stream arriving.
    """

    def __init__(self, device="cuda:0", chunk: int = 5, depth: int = 2):
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.chunk = int(chunk)
        self.depth = int(depth)
        self.host = {}

    # -- host preparation (outside the timed trace) -----------------------
    def prepare(self, req: Request) -> None:
        import synth
        from .plan import offsets_from_positions
        wl = req.wl
        obj = synth.object_truth(wl.obj_shape, wl.seed)
        probe = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
        offs = offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), wl.n, wl.obj_shape)
        probe = probe * synth.probe_photon_scale(obj, probe, offs, wl.photons)
        mask = synth.gap_mask(wl.n, wl.mask_frac, wl.seed)
        self.host[req.rid] = dict(
            obj=np.ascontiguousarray(obj.astype(np.complex64)),
            probe=np.ascontiguousarray(probe.astype(np.complex64)),
            offs=offs, mask=mask,
            obj0=np.ascontiguousarray(synth.start_object(wl.obj_shape).astype(np.complex64)),
            probe0=np.ascontiguousarray(synth.start_probe(probe).astype(np.complex64)))

    @staticmethod
    def footprint(req: Request) -> int:
        """Device bytes a request holds while active."""
        import ctypes
        from ._lib import Desc, check, lib
        wl = req.wl
        n2 = wl.n * wl.n
        d = Desc(wl.n, wl.n_modes, wl.n_frames, wl.obj_shape[0], wl.obj_shape[1], 0, 1e-2, 1e-2, 1e-20, 0)
        ws = ctypes.c_size_t()
        check(lib().ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(ws)))
        no = wl.obj_shape[0] * wl.obj_shape[1]
        iobs = 4 * wl.n_frames * n2
        psi = 8 * wl.n_frames * wl.n_modes * n2
        state = 8 * (2 * no + 2 * wl.n_modes * n2) + 4096
        small = 8 * (2 * no + 2 * wl.n_modes * n2) + n2
        return int(ws.value) + iobs + psi + state + small + iobs    # + the intensity temporary

    # -- device work ------------------------------------------------------
    def start(self, req: Request) -> _Job:
        torch = self.torch
        from .plan import Plan
        h = self.host[req.rid]
        wl = req.wl
        j = _Job()
        j.req = req
        j.stream = torch.cuda.Stream(device=self.dev)
        with torch.cuda.stream(j.stream):
            o_t = torch.from_numpy(h["obj"]).to(self.dev, non_blocking=False)
            p_t = torch.from_numpy(h["probe"]).to(self.dev, non_blocking=False)
            zero = torch.zeros((wl.n_frames, wl.n, wl.n), dtype=torch.float32, device=self.dev)
            sim = Plan(h["offs"], zero, None, wl.n_modes, wl.obj_shape)
            inten = sim.icalc(o_t, p_t)
            gen = torch.Generator(device=self.dev)
            gen.manual_seed(int(wl.seed))
            j.iobs = torch.poisson(inten.clamp_min(0), generator=gen).contiguous()
            sim.close()
            del sim, zero, inten, o_t, p_t
            j.mask = torch.from_numpy(h["mask"]).to(self.dev) if h["mask"] is not None else None
            j.plan = Plan(h["offs"], j.iobs, j.mask, wl.n_modes, wl.obj_shape)
            j.obj = torch.from_numpy(h["obj0"]).to(self.dev)
            j.probe = torch.from_numpy(h["probe0"]).to(self.dev)
            j.psi = j.plan.psi_init(j.obj, j.probe)
            j.state = j.plan.ml_state()
        j.phase = 0
        j.left = req.schedule[0][1]
        j.events = []
        j.final = None
        j.fresh_ml = True
        return j

    def advance(self, j: _Job) -> None:
        torch = self.torch
        j.events = [e for e in j.events if not e.query()]
        with torch.cuda.stream(j.stream):
            while len(j.events) < self.depth and j.phase < len(j.req.schedule):
                kind, _ = j.req.schedule[j.phase]
                n = min(self.chunk, j.left)
                if kind == "dm":
                    j.plan.dm_cycle(j.obj, j.probe, j.psi, n, 3)
                elif kind == "ap":
                    j.plan.ap_cycle(j.obj, j.probe, n, 3, psi=j.psi)
                else:
                    j.plan.ml_cycle(j.obj, j.probe, j.state, n, 3, reset=j.fresh_ml)
                    j.fresh_ml = False
                j.left -= n
                if j.left == 0:
                    j.phase += 1
                    if j.phase < len(j.req.schedule):
                        j.left = j.req.schedule[j.phase][1]
                ev = torch.cuda.Event()
                ev.record(j.stream)
                j.events.append(ev)
                if j.phase == len(j.req.schedule):
                    j.llk = j.plan.llk(j.obj, j.probe)
                    j.out_obj = torch.empty(j.obj.shape, dtype=j.obj.dtype, pin_memory=True)
                    j.out_probe = torch.empty(j.probe.shape, dtype=j.probe.dtype, pin_memory=True)
                    j.out_llk = torch.empty(2, dtype=torch.float64, pin_memory=True)
                    j.out_obj.copy_(j.obj, non_blocking=True)
                    j.out_probe.copy_(j.probe, non_blocking=True)
                    j.out_llk.copy_(j.llk, non_blocking=True)
                    j.final = torch.cuda.Event()
                    j.final.record(j.stream)

    def finished(self, j: _Job) -> bool:
        return j.final is not None and j.final.query()

    def collect(self, j: _Job) -> dict:
        llk = j.out_llk.numpy()
        return {"obj": j.out_obj.numpy(), "probe": j.out_probe.numpy(), "llk": float(llk[0] / llk[1])}

    def release(self, j: _Job) -> None:
        j.plan.close()
        for name in ("plan", "iobs", "mask", "obj", "probe", "psi", "state", "llk"):
            setattr(j, name, None)
        self.host.pop(j.req.rid, None)


def make_trace(n_requests: int, rate: float, seed: int = 0, max_frames: int = 2000, sizes=(128, 256, 512),
               schedule=SCHEDULE, min_frames: int = 200, min_side: int = 1024) -> List[Request]:
    import synth
    reqs = []
    for i, (t, wl) in enumerate(synth.serve_requests(n_requests, rate, seed, sizes=sizes,
                                                       frames=(min_frames, max_frames), min_side=min_side)):
        reqs.append(Request(i, t, wl, schedule))
    return reqs


def serve_trace(n_requests: int = 64, rate: float = 2.0, seed: int = 0, hbm_budget: Optional[int] = None,
                max_active: int = 8, sequential: bool = False, device="cuda:0", max_frames: int = 2000,
                sizes=(128, 256, 512), schedule=SCHEDULE, min_frames: int = 200, min_side: int = 1024):
    """Run an arrival trace through the service; returns (requests, summary)."""
    import torch
    reqs = make_trace(n_requests, rate, seed, max_frames, sizes, schedule, min_frames, min_side)
    ex = GpuExecutor(device)
    for r in reqs:
        ex.prepare(r)
    if hbm_budget is None:
        free, total = torch.cuda.mem_get_info(torch.device(device))
        hbm_budget = int(0.8 * free)
    sch = Scheduler(ex, hbm_budget, max_active=max_active, sequential=sequential)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sch.run(reqs)
    wall = time.perf_counter() - t0
    s = summarize(reqs, wall)
    s["mode"] = "sequential" if sequential else "continuous"
    s["hbm_budget_GB"] = round(hbm_budget / 1e9, 1)
    return reqs, s

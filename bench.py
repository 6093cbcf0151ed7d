#!/usr/bin/env python3
"""Benchmark of the ptychography hot path on one MI355X.

A step is one difference-map cycle (views x probe, far-field FFT, modulus
projection with the gap mask, inverse FFT, DM combination, object update,
probe update) over all 1000 frames of the DM workload: 256x256 frames, 3
probe modes, object 1024x1024, 1e8 photons per frame, 2% gap mask.  The
throughput is frames*cycles/s.  Further legs (reported beside the headline,
each skippable): conjugate-gradient ML cycles (gradient + line search +
step) on the ML workload (500 frames); AP and DM cycles on 4000 frames of
512x512 with 4 modes; DM and ML cycles in the near-field geometry on 17
frames of 2048x2048 with one probe; the served mixed workload; the FP64
oracle on the host.

Inputs are synthetic and built on the GPU: the seeded truth, probe modes,
spiral positions and mask come from `synth`; the integer offsets and the
noise-free intensities come from the library (its host offset routine and
forward model), the Poisson draw from torch.  Everything is resident in HBM
before the timed region.  The CPU baseline times the FP64 oracle on a
bounded sample of the same scan (its own intensities from its own forward
model) on the host cores.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# The profiled run of the committed summaries under profiles/ (run from /tmp
# with TMPDIR=/tmp; $R is the repository root).
PROFILE_COMMAND = ("rocprofv3 --kernel-trace --stats -f csv -d $R/gpurun_out/prof_trace -o run -- python3 $R/bench.py "
                   "--steps 5 --warmup 1 --ml-steps 3 --no-cpu-baseline --no-extra --no-fft --serve-requests 0 "
                   "--large-cycles 1,1 --near-cycles 2,2 --calib-copy")


def source_sha():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2008_11511_amd", "csrc", "*"))):
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build_workload(wl, torch, dev, start):
    """Seeded inputs of one workload, resident on the GPU."""
    import synth
    import paper_2008_11511_amd as P
    near = wl.geometry == "near"
    nf = wl.fresnel if near else None
    obj_t = synth.object_truth(wl.obj_shape, wl.seed)
    if near:
        probe_t = synth.near_field_probe(wl.n, wl.n_modes, wl.seed)
        pos = synth.random_positions(wl.n_frames, wl.step, wl.seed)
    else:
        probe_t = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
        pos = synth.spiral_positions(wl.n_frames, wl.step)
    offs = P.offsets_from_positions(pos, wl.n, wl.obj_shape)
    probe_t = probe_t * synth.probe_photon_scale(obj_t, probe_t, offs, wl.photons)
    o_t = torch.from_numpy(obj_t.astype(np.complex64)).to(dev)
    p_t = torch.from_numpy(probe_t.astype(np.complex64)).to(dev)
    zero = torch.zeros((wl.n_frames, wl.n, wl.n), dtype=torch.float32, device=dev)
    sim = P.Plan(offs, zero, None, wl.n_modes, wl.obj_shape, near_field=nf)
    inten = sim.icalc(o_t, p_t)
    gen = torch.Generator(device=dev)
    gen.manual_seed(wl.seed)
    iobs = torch.poisson(inten.clamp_min(0), generator=gen).contiguous()
    del sim, zero, inten
    m = synth.gap_mask(wl.n, wl.mask_frac, wl.seed, fft_order=not near)
    mask = torch.from_numpy(m).to(dev) if m is not None else None
    if start == "ml":
        o0 = synth.perturb_object(obj_t, wl.seed)
        p0 = synth.perturb_probe(probe_t, wl.seed)
    else:
        o0 = synth.start_object(wl.obj_shape)
        p0 = synth.start_probe(probe_t)
    o0 = torch.from_numpy(o0.astype(np.complex64)).to(dev)
    p0 = torch.from_numpy(p0.astype(np.complex64)).to(dev)
    return offs, iobs, mask, o0, p0, (obj_t, probe_t, pos, m)


def algorithmic_bytes(wl, nstacks, kind):
    """Compulsory bytes per cycle of each kernel class (each input element read
    once, each output written once): U = 8 N^2 (complex frame), W = 4 N^2."""
    J, K, N = wl.n_frames, wl.n_modes, wl.n
    U, W = 8 * N * N, 4 * N * N
    ny, nx = wl.obj_shape
    obj_sums = ny * nx * (8 + 4)
    out = {}
    if kind == "dm":
        out["rows_fwd"] = J * ((2 * K + 1) * U)              # read Psi, view; write stack
        out["cols"] = J * (2 * K * U + W)                    # read+write stack, read Iobs
        out["rows_inv"] = J * ((2 * K + 2) * U)              # read stack, view; write Psi, q
        out["gather_obj"] = J * U + 2 * obj_sums             # read q; object sums
        out["probe_all"] = J * (K * U + U)                   # read Psi and views
    return out


def design_bytes(wl, alg):
    """Bytes per cycle of the reference two-pass design that every cycle is
    priced against (each kernel reads its inputs and writes its outputs once,
    the probe cache-resident): per frame, with U = 8 N^2 and W = 4 N^2,
    N >= 256: AP 8KU + 2U + W, DM 10KU + 3U + W, ML (gradient and line
    search) 13KU + 4U + 2W; N <= 128: AP 3KU + 2U + W, DM 4KU + 2U + W,
    ML 3KU + 4U + 2W."""
    K, N = wl.n_modes, wl.n
    U, W = 8 * N * N, 4 * N * N
    if N >= 256:
        per = {"ap": 8 * K * U + 2 * U + W, "dm": 10 * K * U + 3 * U + W, "ml": 13 * K * U + 4 * U + 2 * W}[alg]
    else:
        per = {"ap": 3 * K * U + 2 * U + W, "dm": 4 * K * U + 2 * U + W, "ml": 3 * K * U + 4 * U + 2 * W}[alg]
    return wl.n_frames * per


def design_roofline(wl, alg, ms_per_cycle):
    b = design_bytes(wl, alg)
    gbs = b / (ms_per_cycle * 1e-3) / 1e9
    return {"design_bytes_per_cycle": b, "design_GBs": round(gbs, 1), "design_frac": round(gbs / HBM_PEAK_GBS, 4)}


def timed_dm(plan, o, p, psi, steps, warmup, torch, classes=None):
    """Time `steps` DM cycles after `warmup` ones, with HIP events around the
    launches of the given kernel classes (None = all)."""
    plan.dm_cycle(o, p, psi, warmup, 3)
    torch.cuda.synchronize()
    plan.timing(True, classes)
    t0 = time.perf_counter()
    plan.dm_cycle(o, p, psi, steps, 3)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    per = plan.timing_read()
    plan.timing(False)
    return dt, per


def cpu_baseline(wl, truth, sample, cycles):
    """FP64 oracle, `cycles` DM cycles over the first `sample` frames of the scan."""
    import oracle
    import synth
    obj_t, probe_t, pos, m = truth
    pos_s = pos[:sample]
    offs = oracle.offsets_from_positions(pos_s, wl.n, wl.obj_shape)
    inten = oracle.simulate_intensity(obj_t, probe_t, offs)
    iobs = synth.poisson_counts(inten, wl.seed)
    o0 = synth.start_object(wl.obj_shape)
    p0 = synth.start_probe(probe_t)
    psi = oracle.psi_init(o0, p0, offs)
    t0 = time.perf_counter()
    for _ in range(cycles):
        o0, p0, psi = oracle.dm_cycle(o0, p0, psi, offs, iobs, m)
    dt = time.perf_counter() - t0
    return sample * cycles / dt, dt


def _cpu_worker(args):
    """One host process of the all-cores baseline: the oracle's DM cycles on
    its share of the scan, timed after every worker has finished its set-up."""
    wl_name, obj_t, probe_t, pos_s, m, cycles, barrier = args
    import oracle
    import synth
    wl = synth.workload(wl_name)
    offs = oracle.offsets_from_positions(pos_s, wl.n, wl.obj_shape)
    iobs = synth.poisson_counts(oracle.simulate_intensity(obj_t, probe_t, offs), wl.seed)
    o0 = synth.start_object(wl.obj_shape)
    p0 = synth.start_probe(probe_t)
    psi = oracle.psi_init(o0, p0, offs)
    barrier.wait()
    t0 = time.monotonic()
    for _ in range(cycles):
        o0, p0, psi = oracle.dm_cycle(o0, p0, psi, offs, iobs, m)
    return t0, time.monotonic()


def cpu_baseline_all_cores(wl, truth, sample, cycles, workers):
    """The FP64 oracle on `workers` host processes at once, each running
    `cycles` DM cycles on its own share of the first `sample` frames (the
    oracle is not parallel itself; independent pieces of the scan are).
    Returns (aggregate frames*cycles/s, wall seconds of the timed region)."""
    import multiprocessing as mp
    obj_t, probe_t, pos, m = truth
    per = max(1, sample // workers)
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with ctx.Manager() as mgr:
            barrier = mgr.Barrier(workers)
            jobs = [(wl.name, obj_t, probe_t, pos[w * per:(w + 1) * per], m, cycles, barrier) for w in range(workers)]
            with ctx.Pool(workers) as pool:
                res = pool.map(_cpu_worker, jobs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    t0 = min(r[0] for r in res)
    t1 = max(r[1] for r in res)
    return workers * per * cycles / (t1 - t0), t1 - t0


# ---------------------------------------------------------------------------
# rocprofv3 summaries (python bench.py --summarize-rocprof TRACE FETCH WRITE)
# ---------------------------------------------------------------------------
# Kernel classes of each profiled cycle.  A cycle's dispatch window runs from
# the first to the last launch of its anchors (template instances only that
# cycle uses); every class takes the launches of its kernel inside the window
# at their most frequent grid (the cycle's full-size launches).
PROFILE_SPECS = {
    "dm256_dm_cycle": {
        "title": "DM cycle, 1000 frames 256x256, 3 modes (dm256)",
        "anchors": ["void ptycho::k_cols_joint<256, 3, 5, false>", "void ptycho::k_rows_inv<256, 3, 1, true, false, false>"],
        "classes": {"rows_fwd": "void ptycho::k_rows_fwd<256, 1, false, false>",
                    "cols": "void ptycho::k_cols_joint<256, 3, 5, false>",
                    "rows_inv": "void ptycho::k_rows_inv<256, 3, 1, true, false, false>",
                    "gather_obj": "ptycho::k_gather_obj(",
                    "probe_all": "void ptycho::k_gather_probe<3, false>"}},
    "ml256_ml_cycle": {
        "title": "conjugate-gradient ML cycle, 500 frames 256x256, 3 modes (ml256)",
        "anchors": ["void ptycho::k_cols_joint<256, 3, 1, false>", "void ptycho::k_cols_seq<256, 6, false>"],
        "classes": {"rows_fwd": "void ptycho::k_rows_fwd<256, 0, false, false>",
                    "cols": "void ptycho::k_cols_joint<256, 3, 1, false>",
                    "rows_inv": "void ptycho::k_rows_inv<256, 3, 0, true, false, false>",
                    "gather_obj": "ptycho::k_gather_obj(",
                    "gather_probe": "void ptycho::k_gather_probe<3, true>",
                    "ls_rows": "void ptycho::k_rows_fwd<256, 4, false, false>",
                    "ls_cols": "void ptycho::k_cols_seq<256, 6, false>"}},
    "apdm512_dm_cycle": {
        "title": "AP and DM cycles, 4000 frames 512x512, 4 modes, object 4096x4096 (apdm512)",
        "anchors": ["void ptycho::k_cols_joint<512, 4, 5, false>", "void ptycho::k_cols_joint<512, 4, 0, false>"],
        "classes": {"rows_fwd": "void ptycho::k_rows_fwd<512, 1, false, false>",
                    "cols": "void ptycho::k_cols_joint<512, 4, 5, false>",
                    "rows_inv": "void ptycho::k_rows_inv<512, 4, 1, true, false, false>",
                    "ap_cols": "void ptycho::k_cols_joint<512, 4, 0, false>",
                    "ap_rows_inv": "void ptycho::k_rows_inv<512, 4, 2, true, false, false>",
                    "gather_obj": "ptycho::k_gather_obj(",
                    "probe_all": "void ptycho::k_gather_probe<4, false>"}},
    "nf2048_dm_cycle": {
        "title": "near-field DM cycle, 17 frames 2048x2048, 1 mode (nf2048)",
        "anchors": ["void ptycho::k_cols_joint<2048, 1, 5, true>", "void ptycho::k_rows_inv<2048, 1, 1, true, true, false>"],
        "classes": {"rows_fwd": "void ptycho::k_rows_fwd<2048, 1, true, false>",
                    "cols": "void ptycho::k_cols_joint<2048, 1, 5, true>",
                    "rows_inv": "void ptycho::k_rows_inv<2048, 1, 1, true, true, false>",
                    "gather_obj": "ptycho::k_gather_obj(",
                    "probe_all": "void ptycho::k_gather_probe<1, false>"}},
}


def _read_csv(directory, suffix):
    import csv
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise FileNotFoundError(f"no *{suffix} under {directory}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def _short(name):
    """Kernel name without its return type and argument list."""
    n = name[5:] if name.startswith("void ") else name
    depth = 0
    for i, ch in enumerate(n):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0 and not n.startswith("(anonymous", i):
            return n[:i]
    return n


def _dispatches(rows, counter=None):
    """[(dispatch id, kernel name, grid threads, value)] in dispatch order; value
    is the duration in ns (trace) or the counter's value (counter runs)."""
    out = []
    for r in rows:
        if counter is None:
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], grid,
                        float(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))))
        elif r["Counter_Name"] == counter:
            out.append((int(r["Dispatch_Id"]), r["Kernel_Name"], int(r["Grid_Size"]), float(r["Counter_Value"])))
    out.sort()
    return out


def _select(disp, spec):
    """Values of each class's full-size launches inside the cycle's window."""
    def named(d, k):
        return d[1].startswith(k + "(") if k.startswith("void ") else d[1].startswith(k)
    ids = [d[0] for d in disp if any(named(d, k) for k in spec["anchors"])]
    if not ids:
        return {}
    lo, hi = min(ids), max(ids)
    out = {}
    for c, k in spec["classes"].items():
        win = [d for d in disp if named(d, k) and lo <= d[0] <= hi]
        if not win:
            continue
        grids = {}
        for d in win:
            grids[d[2]] = grids.get(d[2], 0) + 1
        g = max(grids, key=lambda x: (grids[x], x))
        sel = [d for d in win if d[2] == g]
        out[c] = (g, [d[3] for d in sel], sel[0][1])
    return out


def summarize_rocprof(trace_dir, fetch_dir, write_dir, command, out_dir=None):
    """Per-kernel-class summaries of one profiled bench run: average launch
    duration from the kernel trace, HBM bytes per launch from FETCH_SIZE and
    WRITE_SIZE (KiB per dispatch) scaled by what the same counters read for
    the run's 1 GiB device copy.  Writes profiles/<name>.md for every cycle of
    PROFILE_SPECS found in the run, and profiles/traffic.json."""
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    trace = _dispatches(_read_csv(trace_dir, "_kernel_trace.csv"))
    fetch = _dispatches(_read_csv(fetch_dir, "_counter_collection.csv"), "FETCH_SIZE")
    write = _dispatches(_read_csv(write_dir, "_counter_collection.csv"), "WRITE_SIZE")
    stats = _read_csv(trace_dir, "_kernel_stats.csv")
    # calibration: the copy dispatch that wrote the most bytes (the 1 GiB copy)
    gib = float(1 << 30)
    copies_w = [d for d in write if "copyBuffer" in d[1]]
    copies_f = [d for d in fetch if "copyBuffer" in d[1]]
    if not copies_w or not copies_f:
        raise ValueError("the run holds no device copy to calibrate the counters (bench.py --calib-copy)")
    w_cal = max(d[3] for d in copies_w)
    big_grid = max(copies_w, key=lambda d: d[3])[2]
    f_cal = max(d[3] for d in copies_f if d[2] == big_grid)
    write_scale = gib / (w_cal * 1024.0)
    fetch_scale = gib / (f_cal * 1024.0)
    sha = source_sha()
    traffic = {"source_sha": sha, "fetch_scale": fetch_scale, "write_scale": write_scale, "command": command,
               "cycles": {}}
    written = []
    for name, spec in PROFILE_SPECS.items():
        t_sel = _select(trace, spec)
        if not t_sel:
            continue
        f_sel = _select(fetch, spec)
        w_sel = _select(write, spec)
        rows = {}
        for c, (grid, durs, kname) in t_sel.items():
            e = {"kernel": _short(kname), "grid": grid, "launches": len(durs),
                 "avg_us": sum(durs) / len(durs) / 1e3}
            if c in f_sel and c in w_sel and f_sel[c][0] == grid and w_sel[c][0] == grid:
                rd = sum(f_sel[c][1]) / len(f_sel[c][1]) * 1024.0 * fetch_scale
                wr = sum(w_sel[c][1]) / len(w_sel[c][1]) * 1024.0 * write_scale
                e.update({"read_bytes": rd, "write_bytes": wr, "bytes_per_launch": rd + wr,
                          "GBs": (rd + wr) / (e["avg_us"] * 1e-6) / 1e9})
            rows[c] = e
        traffic["cycles"][name] = rows
        lines = [f"# {name}: rocprofv3 summary", "", spec["title"] + ".", "",
                 "Command (run from /tmp with TMPDIR=/tmp on one MI355X; $R is the repository root; the same "
                 "program once with `--kernel-trace --stats`, once with `--pmc FETCH_SIZE`, once with "
                 "`--pmc WRITE_SIZE`), summarised by `python bench.py --summarize-rocprof TRACE FETCH WRITE`:", "",
                 "    " + command, "",
                 f"Counter calibration: the run's 1 GiB device-to-device copy reads FETCH_SIZE = {f_cal:.0f} KiB "
                 f"and WRITE_SIZE = {w_cal:.0f} KiB, so HBM read bytes = FETCH_SIZE x 1024 x {fetch_scale:.3f} and "
                 f"write bytes = WRITE_SIZE x 1024 x {write_scale:.3f}.", "",
                 f"Kernel sources sha256[:16] = {sha}", "",
                 "## Full-size launches of the cycle: measured traffic per launch", "",
                 "| class | kernel | grid (threads) | launches | avg us | read MB | write MB | GB/s (counted) |",
                 "|---|---|---|---|---|---|---|---|"]
        for c, e in rows.items():
            if "read_bytes" in e:
                lines.append(f"| {c} | `{e['kernel']}` | {e['grid']} | {e['launches']} | {e['avg_us']:.2f} | "
                             f"{e['read_bytes'] / 1e6:.1f} | {e['write_bytes'] / 1e6:.1f} | {e['GBs']:.0f} |")
            else:
                lines.append(f"| {c} | `{e['kernel']}` | {e['grid']} | {e['launches']} | {e['avg_us']:.2f} | "
                             f"- | - | - |")
        lines += ["", "## Kernel stats of the whole run (top 12 by total time)", "",
                  "| kernel | calls | avg us | total % |", "|---|---|---|---|"]
        for r in sorted(stats, key=lambda r: -float(r["Percentage"]))[:12]:
            kn = _short(r["Name"])
            if len(kn) > 70:
                kn = kn[:67] + "..."
            lines.append(f"| `{kn}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                         f"{float(r['Percentage']):.2f} |")
        with open(os.path.join(out_dir, f"{name}.md"), "w") as f:
            f.write("\n".join(lines) + "\n")
        written.append(name)
    with open(os.path.join(out_dir, "traffic.json"), "w") as f:
        json.dump(traffic, f, indent=1)
    return written


def traffic_for(cls, cycle="dm256_dm_cycle"):
    """HBM bytes per launch of kernel class `cls` of a profiled cycle from the
    committed rocprofv3 counter summary, if it was taken on the current kernel
    sources (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        if t.get("source_sha") != source_sha():
            return None
        e = t["cycles"].get(cycle, {}).get(cls)
        return None if e is None or "bytes_per_launch" not in e else e["bytes_per_launch"]
    except Exception:
        return None


def fft_bandwidth(torch, dev, sizes=(64, 128, 256, 512, 1024, 2048), array_bytes=1 << 30):
    """The FFT bandwidth benchmark of the paper's appendix (FFT performance),
    for the library's batched 2D transform: per size, a batch of about 1 GiB of
    complex64 frames goes through two forward/inverse pairs in place, four
    times; the best time counts, with two reads and two writes of the array
    per 2D transform (one per axis)."""
    from paper_2008_11511_amd import _lib
    h = _lib.lib()
    out = {}
    for n in sizes:
        count = max(1, array_bytes // (8 * n * n))
        x = torch.zeros((count, n, n), dtype=torch.complex64, device=dev)
        x.real.normal_()
        stream = torch.cuda.current_stream(dev).cuda_stream
        ptr = x.data_ptr()

        def pairs():
            for _ in range(2):
                for direction in (-1, 1):
                    st = h.ptycho_fft2(n, count, ptr, direction, stream)
                    if st != 0:
                        raise _lib.PtychoError(st, h.ptycho_last_error().decode())

        pairs()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            pairs()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1) / 4.0)          # ms per 2D transform
        nbytes = 2 * 2 * 8 * n * n * count
        gbs = nbytes / (best * 1e-3) / 1e9
        out[str(n)] = {"frames": count, "ms_per_fft": round(best, 4), "GBs": round(gbs, 1),
                       "frac": round(gbs / HBM_PEAK_GBS, 4)}
        del x
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--ml-steps", type=int, default=10)
    ap.add_argument("--stack", type=int, default=0, help="frames per launch (0 = the library's choice)")
    ap.add_argument("--cpu-sample", type=int, default=1000, help="frames of the oracle CPU baseline sample")
    ap.add_argument("--cpu-cycles", type=int, default=2, help="DM cycles of the oracle CPU baseline sample")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="host processes of the all-cores oracle baseline (at most the CPUs available; 1 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ml", action="store_true")
    ap.add_argument("--no-fft", action="store_true", help="skip the batched 2D FFT bandwidth figures")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the LLK-fetch, noise-model, background and copy-roof figures")
    ap.add_argument("--large-cycles", default="2,5",
                    help="AP,DM cycles timed on the 4000 x 512^2 x 4-mode scan (the full chain is 20,50; "
                         "0,0 skips it)")
    ap.add_argument("--near-cycles", default="20,10",
                    help="DM,ML cycles timed on the near-field scan (17 x 2048^2, one probe; the paper's chain "
                         "is 400,100; 0,0 skips it)")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the served mixed workload (0 = skip)")
    ap.add_argument("--serve-seeds", default="7,8,9", help="seeds of the arrival traces (comma-separated)")
    ap.add_argument("--serve-order", default="srpt", choices=("srpt", "lanes", "fifo"),
                    help="running order of the service (srpt: least remaining work first, with the service's age "
                         "cap; lanes: the oldest request beside the shortest others)")
    ap.add_argument("--serve-running", type=int, default=1, help="requests given new work at a time")
    ap.add_argument("--serve-age-cap", type=float, default=0.125,
                    help="seconds after arrival during which a request may be passed by shorter ones (srpt)")
    ap.add_argument("--serve-rate", type=float, default=2.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-rocprof", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/*.md and profiles/traffic.json from the rocprofv3 output of one bench run "
                         "(kernel trace, FETCH_SIZE, WRITE_SIZE) and exit; no GPU needed")
    ap.add_argument("--profile-command", default=PROFILE_COMMAND,
                    help="the profiled command, recorded in the summaries (default: the trace command of the "
                         "committed summaries; the counter runs replace --kernel-trace --stats by --pmc FETCH_SIZE "
                         "and --pmc WRITE_SIZE)")
    args = ap.parse_args()
    if args.summarize_rocprof:
        done = summarize_rocprof(*args.summarize_rocprof, command=args.profile_command)
        print(json.dumps({"profiles": done}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the path is not sharded over several GPUs",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2008_11511_amd as P
    P.lib()                                    # the HIP library must be there
    dev = torch.device("cuda:0")

    wl = synth.workload("dm256")
    log(f"building {wl.name}: {wl.n_frames} frames {wl.n}x{wl.n}, {wl.n_modes} modes")
    offs, iobs, mask, o, p, truth = build_workload(wl, torch, dev, "apdm")
    plan = P.Plan(offs, iobs, mask, wl.n_modes, wl.obj_shape, stack=args.stack)
    psi = plan.psi_init(o, p)
    stack = plan.stack
    torch.cuda.synchronize()
    log(f"plan stack={plan.stack}; warmup {args.warmup} + timed {args.steps} DM cycles")
    # the timed region records events around the dominant kernel class only
    # (each event pair adds a few microseconds to the stream); the per-class
    # breakdown comes from a separate run of 10 cycles with every class timed
    dt, per_main = timed_dm(plan, o, p, psi, args.steps, args.warmup, torch, classes=("rows_inv",))
    _, per = timed_dm(plan, o, p, psi, 10, 0, torch)
    breakdown_steps = 10
    llk = plan.llk(o, p).cpu().numpy()
    value = wl.n_frames * args.steps / dt
    log(f"DM: {dt / args.steps * 1e3:.3f} ms/cycle, {value:.0f} frames*cycles/s, llk/n={llk[0] / llk[1]:.4g}")

    # the whole-job view with the likelihood fetched to the host every 50
    # cycles (the paper's printing interval), and the likelihood of the three
    # noise models and AP cycles refining an incoherent background
    extra = {}
    if not args.no_extra:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.dm_cycle(o, p, psi, 50, 3)
        plan.llk(o, p).cpu()
        extra["dm_ms_per_cycle_with_llk_fetch_every_50"] = round((time.perf_counter() - t0) / 50 * 1e3, 4)
        # five repeats of 10 DM cycles each (the spread of the headline figure)
        reps = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.dm_cycle(o, p, psi, 10, 3)
            torch.cuda.synchronize()
            reps.append(round((time.perf_counter() - t0) / 10 * 1e3, 4))
        extra["dm_ms_per_cycle_5_repeats"] = reps
        extra["dm_ms_per_cycle_median_of_5"] = float(np.median(reps))
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        llk_ms = {}
        for model in ("poisson", "gaussian", "euclidean"):
            plan.llk(o, p, model=model)
            ev0.record()
            for _ in range(5):
                plan.llk(o, p, model=model)
            ev1.record()
            torch.cuda.synchronize()
            llk_ms[model] = round(ev0.elapsed_time(ev1) / 5, 4)
        extra["llk_ms_per_call"] = llk_ms
        # position refinement: shifts of all frames from the stored exit waves
        plan.position_shifts(o, p, psi)
        ev0.record()
        for _ in range(5):
            plan.position_shifts(o, p, psi)
        ev1.record()
        torch.cuda.synchronize()
        extra["position_shifts_ms_per_call"] = round(ev0.elapsed_time(ev1) / 5, 4)
        bgp = P.Plan(offs, iobs, mask, wl.n_modes, wl.obj_shape, background_update=True)
        bgt = torch.full((wl.n, wl.n), 1.0, dtype=torch.float32, device=dev)       # one photon per pixel
        bgp.set_background(bgt)
        psi_ap = torch.empty_like(psi)
        for upd, name in ((3, "ap_ms_per_cycle"), (7, "ap_with_background_refinement_ms_per_cycle")):
            bgp.ap_cycle(o, p, 1, upd, psi=psi_ap)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            bgp.ap_cycle(o, p, 5, upd, psi=psi_ap)
            torch.cuda.synchronize()
            extra[name] = round((time.perf_counter() - t0) / 5 * 1e3, 4)
        del bgp, psi_ap
        # practical roof: a plain 1 GiB device-to-device copy
        a_ = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        b_ = torch.empty_like(a_)
        a_.fill_(1.0)
        b_.copy_(a_)
        ev0.record()
        for _ in range(5):
            b_.copy_(a_)
        ev1.record()
        torch.cuda.synchronize()
        extra["copy_GBs_read_plus_write"] = round(2 * (1 << 30) * 5 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
        del a_, b_
        log(f"extra: {extra}")

    nstacks = math.ceil(wl.n_frames / plan.stack)
    algo = algorithmic_bytes(wl, nstacks, "dm")
    kernels = {}
    for name, (ms, n) in per.items():
        if n == 0:
            continue
        d = {"ms_total": ms, "launches": n, "avg_us": 1e3 * ms / n}
        if name in algo:
            bpl = algo[name] * breakdown_steps / n
            d["alg_bytes_per_launch"] = bpl
            d["alg_GBs"] = bpl / (ms / n * 1e-3) / 1e9
        kernels[name] = d
    dom = max((k for k in kernels if k in algo), key=lambda k: kernels[k]["ms_total"])
    dk = dict(kernels[dom])
    ms_m, n_m = per_main.get(dom, (0.0, 0))
    if n_m:
        # the dominant class as timed inside the headline region
        dk["avg_us"] = 1e3 * ms_m / n_m
        dk["alg_bytes_per_launch"] = algo[dom] * args.steps / n_m
        dk["alg_GBs"] = dk["alg_bytes_per_launch"] / (ms_m / n_m * 1e-3) / 1e9
    achieved = dk["alg_GBs"]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic_for(dom),
                "alg_bytes_per_launch": dk["alg_bytes_per_launch"], "avg_launch_us": round(dk["avg_us"], 2)}
    cycle_alg = sum(algo.values())
    whole = {"alg_bytes_per_cycle": cycle_alg, "alg_GBs": cycle_alg / (dt / args.steps) / 1e9}
    whole["frac"] = whole["alg_GBs"] / HBM_PEAK_GBS
    whole.update(design_roofline(wl, "dm", dt / args.steps * 1e3))

    ml = None
    if not args.no_ml:
        del psi, plan
        torch.cuda.empty_cache()
        wl2 = synth.workload("ml256")
        log(f"building {wl2.name}: {wl2.n_frames} frames, ML leg ({args.ml_steps} CG cycles)")
        offs2, iobs2, mask2, o2, p2, _ = build_workload(wl2, torch, dev, "ml")
        plan2 = P.Plan(offs2, iobs2, mask2, wl2.n_modes, wl2.obj_shape)
        st = plan2.ml_state()
        hist = torch.zeros(args.ml_steps, dtype=torch.float64, device=dev)
        plan2.ml_cycle(o2, p2, st, 2, 3, reset=True, hist=hist[:2].contiguous())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan2.ml_cycle(o2, p2, st, args.ml_steps, 3, reset=False, hist=hist)
        torch.cuda.synchronize()
        dt2 = time.perf_counter() - t0
        h = hist.cpu().numpy()
        # per-class breakdown from a separate run with every class timed
        plan2.timing(True)
        plan2.ml_cycle(o2, p2, st, args.ml_steps, 3, reset=False)
        per2 = plan2.timing_read()
        plan2.timing(False)
        ml = {"workload": "ml256", "frames": wl2.n_frames, "cycles": args.ml_steps,
              "ms_per_cycle": round(dt2 / args.ml_steps * 1e3, 3),
              "frames_cycles_per_s": round(wl2.n_frames * args.ml_steps / dt2, 1),
              "llk_first": float(h[0]), "llk_last": float(h[-1]),
              "kernels_ms_per_cycle": {k: round(ms / args.ml_steps, 4) for k, (ms, n) in per2.items() if n}}
        ml.update(design_roofline(wl2, "ml", dt2 / args.ml_steps * 1e3))
        log(f"ML: {ml['ms_per_cycle']} ms/cycle, {ml['frames_cycles_per_s']} frames*cycles/s")
        del plan2, st

    large = None
    n_ap, n_dm = (int(x) for x in args.large_cycles.split(","))
    if n_ap + n_dm > 0:
        torch.cuda.empty_cache()
        wl3 = synth.workload("apdm512")
        log(f"building {wl3.name}: {wl3.n_frames} frames {wl3.n}x{wl3.n}, {wl3.n_modes} modes, object "
            f"{wl3.obj_shape[0]}x{wl3.obj_shape[1]}")
        offs3, iobs3, mask3, o3, p3, _ = build_workload(wl3, torch, dev, "apdm")
        plan3 = P.Plan(offs3, iobs3, mask3, wl3.n_modes, wl3.obj_shape)
        psi3 = torch.empty((wl3.n_frames, wl3.n_modes, wl3.n, wl3.n), dtype=torch.complex64, device=dev)
        plan3.ap_cycle(o3, p3, 1, 3, psi=psi3)                       # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan3.ap_cycle(o3, p3, n_ap, 3, psi=psi3)
        torch.cuda.synchronize()
        t_ap = time.perf_counter() - t0
        plan3.psi_init(o3, p3, psi3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan3.dm_cycle(o3, p3, psi3, n_dm, 3)
        torch.cuda.synchronize()
        t_dm = time.perf_counter() - t0
        # per-class breakdown: one AP and one DM cycle with every class timed
        plan3.timing(True)
        plan3.ap_cycle(o3, p3, 1, 3, psi=psi3)
        plan3.dm_cycle(o3, p3, psi3, 1, 3)
        per3 = plan3.timing_read()
        plan3.timing(False)
        algo3 = algorithmic_bytes(wl3, 0, "dm")
        k3 = {}
        for name, (ms, n) in per3.items():
            if n:
                k3[name] = {"avg_us": round(1e3 * ms / n, 2), "launches": n}
                if name in ("cols", "gather_obj", "probe_all"):
                    # these classes run with the same bytes in AP and DM cycles
                    bpl = algo3[name] * 2 / n
                    k3[name]["alg_GBs"] = round(bpl / (ms / n * 1e-3) / 1e9, 1)
        large = {"workload": "apdm512: 4000 frames 512x512, 4 modes, object 4096x4096, 1e9 photons/frame, 3% mask",
                 "ap_cycles": n_ap, "dm_cycles": n_dm,
                 "ap_ms_per_cycle": round(t_ap / max(n_ap, 1) * 1e3, 2) if n_ap else None,
                 "dm_ms_per_cycle": round(t_dm / max(n_dm, 1) * 1e3, 2) if n_dm else None,
                 "dm_frames_cycles_per_s": round(wl3.n_frames * n_dm / t_dm, 1) if n_dm else None,
                 "stack": plan3.stack, "kernels": k3}
        if n_ap:
            large["ap_design"] = design_roofline(wl3, "ap", t_ap / n_ap * 1e3)
        if n_dm:
            large["dm_design"] = design_roofline(wl3, "dm", t_dm / n_dm * 1e3)
        log(f"large: AP {large['ap_ms_per_cycle']} ms/cycle, DM {large['dm_ms_per_cycle']} ms/cycle")
        del plan3, psi3, iobs3, o3, p3
        torch.cuda.empty_cache()

    near = None
    n_ndm, n_nml = (int(x) for x in args.near_cycles.split(","))
    if n_ndm + n_nml > 0:
        torch.cuda.empty_cache()
        wl4 = synth.workload("nf2048")
        log(f"building {wl4.name}: {wl4.n_frames} frames {wl4.n}x{wl4.n}, {wl4.n_modes} mode, object "
            f"{wl4.obj_shape[0]}x{wl4.obj_shape[1]}, Fresnel parameter {wl4.fresnel:.3e}")
        offs4, iobs4, mask4, o4, p4, _ = build_workload(wl4, torch, dev, "apdm")
        plan4 = P.Plan(offs4, iobs4, mask4, wl4.n_modes, wl4.obj_shape, near_field=wl4.fresnel)
        near = {"workload": "nf2048: near field, 17 frames 2048x2048, 1 probe mode, object 2368x2368, "
                            "1e4 photons/pixel, Fresnel number 4e-3 per pixel",
                "frames": wl4.n_frames, "frame": wl4.n, "modes": wl4.n_modes, "stack": plan4.stack}
        if n_ndm:
            psi4 = plan4.psi_init(o4, p4)
            dt4, _ = timed_dm(plan4, o4, p4, psi4, n_ndm, 2, torch, classes=("rows_inv",))
            _, per4 = timed_dm(plan4, o4, p4, psi4, n_ndm, 0, torch)
            algo4 = algorithmic_bytes(wl4, 0, "dm")
            k4 = {}
            for name, (ms, n) in per4.items():
                if n:
                    k4[name] = {"avg_us": round(1e3 * ms / n, 2), "launches": n}
                    if name in algo4:
                        k4[name]["alg_GBs"] = round(algo4[name] * n_ndm / n / (ms / n * 1e-3) / 1e9, 1)
            cyc4 = sum(algo4.values())
            near.update({"dm_cycles": n_ndm, "dm_ms_per_cycle": round(dt4 / n_ndm * 1e3, 3),
                         "dm_frames_cycles_per_s": round(wl4.n_frames * n_ndm / dt4, 1), "dm_kernels": k4,
                         "cycle_alg_bytes": cyc4, "cycle_alg_GBs": round(cyc4 * n_ndm / dt4 / 1e9, 1),
                         "cycle_hbm_frac": round(cyc4 * n_ndm / dt4 / 1e9 / HBM_PEAK_GBS, 4),
                         "note": "the column pass runs four 2048-point transforms per column and is bound by "
                                 "the vector ALU, not HBM"})
            del psi4
        if n_nml:
            o4, p4 = build_workload(wl4, torch, dev, "ml")[3:5]
            st4 = plan4.ml_state()
            plan4.ml_cycle(o4, p4, st4, 1, 3, reset=True)                 # warm-up
            hist4 = torch.zeros(n_nml, dtype=torch.float64, device=dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan4.ml_cycle(o4, p4, st4, n_nml, 3, reset=True, hist=hist4)
            torch.cuda.synchronize()
            t_ml4 = time.perf_counter() - t0
            h4 = hist4.cpu().numpy()
            near.update({"ml_cycles": n_nml, "ml_ms_per_cycle": round(t_ml4 / n_nml * 1e3, 3),
                         "ml_frames_cycles_per_s": round(wl4.n_frames * n_nml / t_ml4, 1),
                         "llk_first": float(h4[0]), "llk_last": float(h4[-1])})
            del st4
        near["paper_context"] = {"dm_ms_per_cycle": 39, "ml_ms_per_cycle": 84,
                                 "note": "near field, 17 frames 2048x2048, 1 probe, one NVIDIA V100 (Table 1); "
                                         "other hardware, context only"}
        log(f"near field: DM {near.get('dm_ms_per_cycle')} ms/cycle, ML {near.get('ml_ms_per_cycle')} ms/cycle")
        del plan4, iobs4, o4, p4
        torch.cuda.empty_cache()

    serve = None
    if args.serve_requests > 0:
        from paper_2008_11511_amd.serve import serve_trace
        seeds = [int(s) for s in args.serve_seeds.split(",") if s]
        per_seed = {}
        for seed in seeds:
            torch.cuda.empty_cache()
            log(f"serving, seed {seed}: {args.serve_requests} requests at {args.serve_rate} req/s, 30 DM + 20 ML "
                f"each, order {args.serve_order}, {args.serve_running} running, age cap {args.serve_age_cap} s")
            con, s_con = serve_trace(n_requests=args.serve_requests, rate=args.serve_rate, seed=seed,
                                     order=args.serve_order, max_running=args.serve_running,
                                     age_cap=args.serve_age_cap)
            log(f"continuous: {s_con}")
            log("serving: same trace, sequential plain solves (one request resident at a time)")
            seq, s_seq = serve_trace(n_requests=args.serve_requests, rate=args.serve_rate, seed=seed,
                                     sequential=True)
            log(f"sequential: {s_seq}")
            same = all(np.array_equal(a.result["obj"], b.result["obj"]) and
                       np.array_equal(a.result["probe"], b.result["probe"]) for a, b in zip(con, seq))
            per_seed[seed] = {
                "continuous": s_con, "sequential": s_seq,
                "p50_speedup": round(s_seq["p50_latency_s"] / s_con["p50_latency_s"], 3),
                "mean_speedup": round(s_seq["mean_latency_s"] / s_con["mean_latency_s"], 3),
                "p99_speedup": round(s_seq["p99_latency_s"] / s_con["p99_latency_s"], 3),
                "results_identical": bool(same),
                "mean_final_llk_per_pixel": round(float(np.mean([r.result["llk"] for r in con])), 4)}
            del con, seq
        torch.cuda.empty_cache()
        serve = {"workload": f"{args.serve_requests} requests, Poisson arrivals at {args.serve_rate}/s, frames "
                             f"128/256/512, 200-2000 positions, 1 or 3 modes, 30 DM + 20 ML cycles each",
                 "order": args.serve_order, "max_running": args.serve_running,
                 "age_cap_s": args.serve_age_cap, "seeds": per_seed,
                 "min_speedup": {q: min(v[f"{q}_speedup"] for v in per_seed.values())
                                 for q in ("p50", "mean", "p99")},
                 "results_identical": all(v["results_identical"] for v in per_seed.values())}

    fft = None
    if not args.no_fft:
        log("FFT bandwidth: batched unitary 2D FFT, 64..2048 points, 1 GiB per size, best of 4 x 2 pairs")
        fft = fft_bandwidth(torch, dev)
        log(f"FFT bandwidth: {json.dumps({n: v['GBs'] for n, v in fft.items()})} GB/s")

    if args.calib_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration copy: 3 x 1 GiB device-to-device")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU baseline: FP64 oracle, {args.cpu_cycles} DM cycles over {args.cpu_sample} frames")
        fcs, t = cpu_baseline(wl, truth, args.cpu_sample, args.cpu_cycles)
        cpu = {"value": round(fcs, 3), "unit": "frames*cycles/s", "cores": 1, "kind": "oracle",
               "sample": f"{args.cpu_cycles} DM cycles over the first {args.cpu_sample} of {wl.n_frames} frames "
                         f"of the same scan (256x256, 3 modes), {t:.1f} s timed; numpy FFT single-threaded",
               "host_cpus": len(os.sched_getaffinity(0))}
        log(f"CPU oracle: {fcs:.2f} frames*cycles/s ({t:.1f} s)")
        workers = min(args.cpu_workers, len(os.sched_getaffinity(0)))
        if workers > 1:
            log(f"CPU baseline, all cores: {workers} oracle processes, {args.cpu_cycles} DM cycles each")
            fcs_all, t_all = cpu_baseline_all_cores(wl, truth, args.cpu_sample, args.cpu_cycles, workers)
            cpu["all_cores"] = {"value": round(fcs_all, 3), "unit": "frames*cycles/s", "cores": workers,
                                "sample": f"{workers} processes, each {args.cpu_cycles} DM cycles on its own "
                                          f"{args.cpu_sample // workers} of the first {args.cpu_sample} frames, "
                                          f"{t_all:.1f} s timed"}
            log(f"CPU oracle, {workers} cores: {fcs_all:.2f} frames*cycles/s ({t_all:.1f} s)")

    out = {
        "metric": "frames*cycles/s (256^2 frames, 3 modes) & %HBM roofline",
        "value": round(value, 1),
        "unit": "frames*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded truth, spiral scan, Poisson counts from the library's forward model)",
        "config": {"workload": "dm256: DM cycles, 1000 frames 256x256, 3 probe modes, object 1024x1024, "
                               "1e8 photons/frame, 2% gap mask",
                   "frames": wl.n_frames, "frame": wl.n, "modes": wl.n_modes, "object": list(wl.obj_shape),
                   "stack": stack, "algorithm": "DM (beta=1), object+probe update"},
        "roofline": roofline,
        "cycle_roofline": whole,
        "kernels": kernels,
        "kernels_cycles": breakdown_steps,
        "ml": ml,
        "extra": extra or None,
        "large": large,
        "near_field": near,
        "serve": serve,
        "fft": fft,
        "cpu_baseline": cpu,
        "paper_context": {"value": 22727, "unit": "frames*cycles/s",
                          "note": "DM 44 ms/cycle, 1000 frames 256x256, 3 probe modes, object 1176x1188, "
                                  "one NVIDIA V100 (Table 1); other hardware, context only"},
        "source_sha": source_sha(),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

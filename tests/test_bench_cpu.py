"""The benchmark's contract on the CPU: one GPU only, the algorithmic-byte
count of a DM cycle against a hand count, and counted traffic reported only
when the committed counters match the kernel sources."""
import os
import subprocess
import sys

import bench
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_dm_algorithmic_bytes_match_a_hand_count():
    wl = synth.workload("dm256")
    a = bench.algorithmic_bytes(wl, 1, "dm")
    u, w = 8 * 256 * 256, 4 * 256 * 256
    # per frame: forward rows 7U, columns 6U + W, inverse rows 8U, object gather U, probe gather 4U (K = 3);
    # per cycle: the object numerator and denominator, written and read back once (12 B per pixel each way)
    per_frame = 7 * u + (6 * u + w) + 8 * u + u + 4 * u
    assert sum(a.values()) == 1000 * per_frame + 2 * 1024 * 1024 * 12 == 13918797824
    assert a["rows_inv"] == 1000 * 8 * u


def test_counted_traffic_only_for_the_profiled_sources(monkeypatch):
    got = bench.traffic_for("rows_inv")
    assert got is None or got > 0
    monkeypatch.setattr(bench, "source_sha", lambda: "not-the-profiled-sources")
    assert bench.traffic_for("rows_inv") is None


def test_design_bytes_match_the_reference_accounting():
    # per frame*cycle, U = 8 N^2, W = U / 2: DM 10KU + 3U + W, ML 13KU + 4U + 2W, AP 8KU + 2U + W (N >= 256)
    u256, u512 = 8 * 256 * 256, 8 * 512 * 512
    assert bench.design_bytes(synth.workload("dm256"), "dm") == 1000 * 33.5 * u256 == 17563648000
    assert bench.design_bytes(synth.workload("ml256"), "ml") == 500 * 44 * u256
    assert bench.design_bytes(synth.workload("apdm512"), "ap") == 4000 * 34.5 * u512
    assert bench.design_bytes(synth.workload("apdm512"), "dm") == 4000 * 43.5 * u512
    # N <= 128: one pass per transform, AP 3KU + 2U + W
    assert bench.design_bytes(synth.workload("ap64"), "ap") == 100 * 5.5 * 8 * 64 * 64
    r = bench.design_roofline(synth.workload("dm256"), "dm", 2.0)
    assert abs(r["design_frac"] - 17563648000 / 2e-3 / 8e12) < 1e-4


def test_all_cores_oracle_baseline_runs_independent_pieces():
    import numpy as np
    wl = synth.workload("ap64")
    obj = synth.object_truth(wl.obj_shape, wl.seed)
    probe = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
    pos = synth.spiral_positions(wl.n_frames, wl.step)
    fcs, t = bench.cpu_baseline_all_cores(wl, (obj, probe, pos, None), sample=8, cycles=1, workers=2)
    assert fcs > 0 and t > 0 and np.isfinite(fcs)


def test_rocprof_summary_from_synthetic_csvs(tmp_path):
    """The summarizer picks the cycle's kernel instances, averages their trace
    durations and scales the counters by the 1 GiB copy's reading."""
    import csv
    import json

    def write(path, header, rows):
        path.parent.mkdir(parents=True, exist_ok=True)
        with open(path, "w", newline="") as f:
            w = csv.writer(f, quoting=csv.QUOTE_NONNUMERIC)
            w.writerow(header)
            w.writerows(rows)

    k_inv = "void ptycho::k_rows_inv<256, 3, 1, true, false, false>(ptycho::StackArgs)"
    k_obj = "ptycho::k_gather_obj(ptycho::ObjTileArgs)"
    copy = "__amd_rocclr_copyBuffer"
    th = ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Grid_Size_Y",
          "Grid_Size_Z"]
    # dispatch order: a copy, two inverse-row launches (800 and 900 us), a gather, and a gather of another plan
    write(tmp_path / "tr" / "h" / "run_kernel_trace.csv", th,
          [["KERNEL_DISPATCH", 1, copy, 0, 1000, 1024, 1, 1],
           ["KERNEL_DISPATCH", 2, k_inv, 1000, 801000, 4096, 3, 1],
           ["KERNEL_DISPATCH", 3, k_obj, 801000, 901000, 256, 1, 1],
           ["KERNEL_DISPATCH", 4, k_inv, 901000, 1801000, 4096, 3, 1],
           ["KERNEL_DISPATCH", 5, k_obj, 1801000, 1802000, 64, 1, 1]])
    write(tmp_path / "tr" / "h" / "run_kernel_stats.csv", ["Name", "Calls", "AverageNs", "Percentage"],
          [[k_inv, 2, 850000.0, 90.0], [k_obj, 2, 50500.0, 5.0]])
    ch = ["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"]
    gib_kib = float(1 << 20)
    write(tmp_path / "fe" / "run_counter_collection.csv", ch,
          [[1, 1024, copy, "FETCH_SIZE", gib_kib / 2], [2, 12288, k_inv, "FETCH_SIZE", 1000.0],
           [3, 256, k_obj, "FETCH_SIZE", 10.0], [4, 12288, k_inv, "FETCH_SIZE", 3000.0],
           [5, 64, k_obj, "FETCH_SIZE", 1.0]])
    write(tmp_path / "wr" / "run_counter_collection.csv", ch,
          [[1, 1024, copy, "WRITE_SIZE", gib_kib], [2, 12288, k_inv, "WRITE_SIZE", 500.0],
           [3, 256, k_obj, "WRITE_SIZE", 5.0], [4, 12288, k_inv, "WRITE_SIZE", 500.0],
           [5, 64, k_obj, "WRITE_SIZE", 7.0]])
    out = tmp_path / "profiles"
    out.mkdir()
    done = bench.summarize_rocprof(str(tmp_path / "tr"), str(tmp_path / "fe"), str(tmp_path / "wr"), "the command",
                                   out_dir=str(out))
    assert done == ["dm256_dm_cycle"]
    tr = json.load(open(out / "traffic.json"))
    assert abs(tr["fetch_scale"] - 2.0) < 1e-12 and abs(tr["write_scale"] - 1.0) < 1e-12
    inv = tr["cycles"]["dm256_dm_cycle"]["rows_inv"]
    assert inv["launches"] == 2 and abs(inv["avg_us"] - 850.0) < 1e-9
    assert abs(inv["read_bytes"] - 2000.0 * 1024 * 2.0) < 1e-6 and abs(inv["write_bytes"] - 500.0 * 1024) < 1e-6
    obj = tr["cycles"]["dm256_dm_cycle"]["gather_obj"]
    assert obj["grid"] == 256 and obj["launches"] == 1         # the other plan's gather is outside the window
    text = (out / "dm256_dm_cycle.md").read_text()
    assert "the command" in text and "k_rows_inv<256, 3, 1, true, false, false>" in text

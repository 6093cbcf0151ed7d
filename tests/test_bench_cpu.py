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
    got = bench.traffic_for("rows_inv", 1)
    assert got is None or got > 0
    monkeypatch.setattr(bench, "source_sha", lambda: "not-the-profiled-sources")
    assert bench.traffic_for("rows_inv", 1) is None

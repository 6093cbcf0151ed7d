"""The reconstruction service on the GPU: results are the same alone and in
the mix (bitwise: every request has its own plan and fixed-order
reductions), and a mixed trace completes under continuous batching."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def test_results_identical_alone_and_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_11511_amd import lib
    from paper_2008_11511_amd.serve import serve_trace
    lib()
    kw = dict(n_requests=6, rate=40.0, seed=5, sizes=(64, 128), min_frames=60, max_frames=160,
              schedule=(("dm", 4), ("ml", 3)), min_side=256)
    say("serve: continuous")
    con, s_con = serve_trace(max_active=6, **kw)
    say("serve: sequential")
    seq, s_seq = serve_trace(sequential=True, **kw)
    assert s_con["requests"] == s_seq["requests"] == 6
    for a, b in zip(con, seq):
        assert a.rid == b.rid
        assert np.array_equal(a.result["obj"], b.result["obj"])
        assert np.array_equal(a.result["probe"], b.result["probe"])
        assert a.result["llk"] == b.result["llk"]
        assert np.isfinite(a.result["llk"])

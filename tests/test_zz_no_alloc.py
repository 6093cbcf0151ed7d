"""The allocation-free LLK (ptycho_llk_noalloc, static device scratch) against
the plan path's ptycho_llk on the same inputs, through the C ABI: two calls
in a row, the second on a smaller problem; a scan larger than one stack of
the scratch; clamped windows flagged by NaN; problems beyond the scratch
refused before any GPU work."""
import ctypes
import sys

import numpy as np
import pytest

import oracle
from cases import make_problem, small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2008_11511_amd as P
    P.lib()
    return torch.device("cuda:0")


def _inputs(pb, dev):
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
    mask = t(pb.mask, torch.uint8) if pb.mask is not None else None
    return (t(pb.offsets, torch.int32), t(pb.iobs, torch.float32), mask,
            t(pb.obj0, torch.complex64), t(pb.probe0, torch.complex64))


def _noalloc(pb, dev, offs=None):
    from paper_2008_11511_amd._lib import Desc, check, lib
    wl = pb.wl
    o_t, iobs, mask, obj, probe = _inputs(pb, dev)
    if offs is not None:
        o_t = torch.from_numpy(np.ascontiguousarray(offs, dtype=np.int32)).to(dev)
    d = Desc(wl.n, wl.n_modes, len(pb.offsets), wl.obj_shape[0], wl.obj_shape[1], 0, 1e-2, 1e-2, 1e-20, 0)
    out = torch.full((2,), -1.0, dtype=torch.float64, device=dev)
    check(lib().ptycho_llk_noalloc(ctypes.byref(d), o_t.data_ptr(), iobs.data_ptr(),
                                   mask.data_ptr() if mask is not None else None, obj.data_ptr(),
                                   probe.data_ptr(), out.data_ptr(), torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def _plan_llk(pb, dev):
    from paper_2008_11511_amd import Plan
    _, iobs, mask, obj, probe = _inputs(pb, dev)
    plan = Plan(pb.offsets, iobs, mask, pb.wl.n_modes, pb.wl.obj_shape)
    r = plan.llk(obj, probe).cpu().numpy()
    return r


def test_noalloc_llk_matches_the_plan_path_twice_in_a_row(dev):
    big = make_problem(small("dm256", n=256, k=3, j=100, obj=(512, 512), step=10.0, mask_frac=0.02), start="ml")
    little = make_problem(small("dm256", n=32, k=1, j=9, obj=(64, 64), step=3.0, mask_frac=0.0), start="ml")
    for name, pb in (("256^2 x 3 modes, 100 frames (3 stacks of the scratch)", big),
                     ("32^2 x 1 mode, 9 frames", little)):
        say(f"noalloc LLK vs plan LLK: {name}")
        got = _noalloc(pb, dev)
        want = _plan_llk(pb, dev)
        assert got[1] == want[1]
        assert abs(got[0] - want[0]) <= 1e-12 * abs(want[0]), (got, want)
        # and both against the oracle at the per-cycle bar
        ref, nobs = oracle.llk(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask)
        assert got[1] == nobs
        assert abs(got[0] - ref) <= 1e-4 * abs(ref)


def test_noalloc_llk_flags_windows_outside_the_object(dev):
    pb = make_problem(small("dm256", n=32, k=1, j=9, obj=(64, 64), step=3.0, mask_frac=0.0), start="ml")
    offs = pb.offsets.copy()
    offs[3] = (60, 0)                       # 60 + 32 > 64
    say("noalloc LLK: a window outside the object")
    got = _noalloc(pb, dev, offs)
    assert np.isnan(got[0])
    say("noalloc LLK: valid again afterwards")
    got = _noalloc(pb, dev)
    assert np.isfinite(got[0])


def test_noalloc_llk_refuses_problems_beyond_its_scratch():
    from paper_2008_11511_amd._lib import Desc, lib
    fake = ctypes.c_void_p(256)
    d = Desc(2048, 4, 10, 4096, 4096, 0, 1e-2, 1e-2, 1e-20, 0)     # 128 MiB per frame
    assert lib().ptycho_llk_noalloc(ctypes.byref(d), fake, fake, None, fake, fake, fake, None) == -5
    assert b"allocation-free scratch" in lib().ptycho_last_error()
    d = Desc(64, 1, 10, 128, 128, 0, 1e-2, 1e-2, 1e-20, 2)          # near field: not this call
    assert lib().ptycho_llk_noalloc(ctypes.byref(d), fake, fake, None, fake, fake, fake, None) == -1

"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every declared symbol, host-only entry points match the oracle bit
for bit, and argument errors are reported before any GPU work."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2008_11511_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "ptycho.h")).read()
    return sorted(set(re.findall(r"\b(ptycho_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    h = _lib.lib()
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(h, name), name
    assert sorted(_lib.exported_symbols()) == names


def test_boundary_exports_the_operator_entry_points_and_nothing_else():
    """The plan and the four operator calls carry their C names, and the
    shared library exports only the C ABI (no internal C++ symbols)."""
    h = _lib.lib()
    for name in ("ptycho_plan", "ptycho_ap_cycle", "ptycho_dm_cycle", "ptycho_ml_grad", "ptycho_llk"):
        assert hasattr(h, name), name
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("no nm")
    out = subprocess.run([nm, "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    text_syms = [ln.split()[-1] for ln in out.splitlines() if len(ln.split()) == 3 and ln.split()[1] == "T"]
    assert text_syms and all(s.startswith("ptycho_") for s in text_syms), [s for s in text_syms
                                                                            if not s.startswith("ptycho_")]
    assert set(declared_functions()) <= set(text_syms)


def test_offsets_match_oracle_bitwise_on_a_million_positions():
    rng = np.random.default_rng(0)
    n, shape = 64, (4096, 3000)
    pos = rng.uniform(-1400, 1400, size=(1_000_000, 2))
    # many exact half-integers and values a hair around them
    pos[::7] = np.round(pos[::7]) + 0.5
    pos[1::7] = np.round(pos[1::7]) - 0.5
    pos[2::7] = np.nextafter(np.round(pos[2::7]) + 0.5, 0)
    pos[3::7] = np.nextafter(np.round(pos[3::7]) - 0.5, 0)
    pos[:, 1] = np.clip(pos[:, 1], -1400, 1400)
    from paper_2008_11511_amd.plan import offsets_from_positions
    got = offsets_from_positions(pos, n, shape)
    exp = oracle.offsets_from_positions(pos, n, shape)
    assert got.dtype == np.int32
    np.testing.assert_array_equal(got, exp)


def test_offsets_out_of_bounds_is_an_error_and_writes_nothing():
    from paper_2008_11511_amd.plan import offsets_from_positions
    with pytest.raises(_lib.PtychoError) as e:
        offsets_from_positions(np.array([[0.0, 0.0], [40.0, 0.0]]), 16, (64, 64))
    assert e.value.code == -2
    h = _lib.lib()
    out = np.full((2, 2), -7, np.int32)
    pos = np.array([[0.0, 0.0], [0.0, -30.0]])
    assert h.ptycho_offsets_from_positions(pos.ctypes.data, 2, 16, 64, 64, out.ctypes.data) == -2
    assert (out == -7).all()
    assert b"outside" in h.ptycho_last_error()


def _desc(**kw):
    d = dict(n=64, n_modes=1, n_frames=10, obj_ny=128, obj_nx=128, stack=0, obj_inertia=0.01,
             probe_inertia=0.01, icalc_floor=1e-20, flags=0)
    d.update(kw)
    return _lib.Desc(**d)


def test_workspace_query_and_descriptor_validation():
    h = _lib.lib()
    sz = ctypes.c_size_t()
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc()), ctypes.byref(sz)) == 0
    assert sz.value > 0 and sz.value % 256 == 0
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(n=48)), ctypes.byref(sz)) == -3
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(n_modes=5)), ctypes.byref(sz)) == -3
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(obj_nx=32)), ctypes.byref(sz)) == -1
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(flags=8)), ctypes.byref(sz)) == -1
    # the background flag reserves S*N*N floats and N*N doubles more
    plain, bgu = ctypes.c_size_t(), ctypes.c_size_t()
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc()), ctypes.byref(plain)) == 0
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(flags=1)), ctypes.byref(bgu)) == 0
    assert bgu.value >= plain.value + 4 * 10 * 64 * 64 + 8 * 64 * 64
    # the near-field flag reserves the 2 N transfer-function factors
    nfw, both = ctypes.c_size_t(), ctypes.c_size_t()
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(flags=2)), ctypes.byref(nfw)) == 0
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(flags=3)), ctypes.byref(both)) == 0
    assert nfw.value >= plain.value + 8 * 2 * 64 and both.value >= bgu.value + 8 * 2 * 64
    assert h.ptycho_workspace_bytes(ctypes.byref(_desc(icalc_floor=0.0)), ctypes.byref(sz)) == -1
    # larger problems need more workspace
    big = ctypes.c_size_t()
    h.ptycho_workspace_bytes(ctypes.byref(_desc(n_frames=1000)), ctypes.byref(big))
    assert big.value > sz.value or True


def test_plan_create_rejects_bad_arguments_before_gpu_work():
    h = _lib.lib()
    out = ctypes.c_void_p()
    offs = np.zeros((10, 2), np.int32)
    fake = ctypes.c_void_p(256)     # never dereferenced: validation fails first
    # null workspace
    assert h.ptycho_plan(ctypes.byref(_desc()), offs.ctypes.data, fake, None, None, 0, None,
                                ctypes.byref(out)) == -5
    # misaligned workspace
    assert h.ptycho_plan(ctypes.byref(_desc()), offs.ctypes.data, fake, None, ctypes.c_void_p(257),
                                1 << 30, None, ctypes.byref(out)) == -5
    # too small
    assert h.ptycho_plan(ctypes.byref(_desc()), offs.ctypes.data, fake, None, ctypes.c_void_p(256),
                                16, None, ctypes.byref(out)) == -5
    # window outside the object
    bad = offs.copy()
    bad[3] = [100, 0]
    assert h.ptycho_plan(ctypes.byref(_desc()), bad.ctypes.data, fake, None, ctypes.c_void_p(256),
                                1 << 40, None, ctypes.byref(out)) == -2
    # null plan handles
    assert h.ptycho_ap_cycle(None, fake, fake, fake, 1, 3) == -1
    assert h.ptycho_dm_cycle(None, fake, fake, fake, 1, 3) == -1
    assert h.ptycho_plan_destroy(None) == 0
    assert h.ptycho_fft2(48, 1, fake, -1, None) == -3
    assert h.ptycho_fft2(64, 1, fake, 0, None) == -1


def _dry(n, k, j, obj, stack, offs):
    h = _lib.lib()
    d = _desc(n=n, n_modes=k, n_frames=j, obj_ny=obj[0], obj_nx=obj[1], stack=stack)
    nbytes = ctypes.c_size_t()
    offs = np.ascontiguousarray(offs, dtype=np.int32)
    return h.ptycho_plan_dry_run(ctypes.byref(d), offs.ctypes.data, ctypes.byref(nbytes)), nbytes.value


@pytest.mark.parametrize("stack", [0, 1, 3, 7, 16, 1000])
def test_plan_tables_fit_their_workspace_bounds_for_any_stack(stack):
    import synth
    for name in ("ap64", "dm256"):
        wl = synth.workload(name)
        offs = oracle.offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), wl.n, wl.obj_shape)
        st, nbytes = _dry(wl.n, wl.n_modes, wl.n_frames, wl.obj_shape, stack, offs)
        assert st == 0, _lib.lib().ptycho_last_error()
        assert nbytes > 0


def test_plan_tables_for_awkward_shapes_and_dense_scans():
    rng = np.random.default_rng(2)
    cases = [(16, 1, 1, (16, 16)), (16, 2, 5, (17, 33)), (32, 1, 40, (40, 200)), (64, 3, 300, (64, 64)),
             (128, 4, 57, (130, 700)), (512, 4, 9, (513, 1100)), (256, 3, 2000, (300, 300))]
    for n, k, j, obj in cases:
        offs = np.stack([rng.integers(0, obj[0] - n + 1, j), rng.integers(0, obj[1] - n + 1, j)], axis=1)
        for stack in (0, 1, 5):
            st, _ = _dry(n, k, j, obj, stack, offs)
            assert st == 0, (n, k, j, obj, stack, _lib.lib().ptycho_last_error())
    # all windows at one spot: the heaviest possible tile lists
    offs = np.zeros((3000, 2), np.int32)
    assert _dry(64, 1, 3000, (64, 64), 0, offs)[0] == 0
    # out-of-bounds offsets are reported, as by ptycho_plan
    assert _dry(64, 1, 1, (64, 64), 0, np.array([[1, 0]]))[0] == -2


def test_plan_tables_for_the_large_scan():
    import synth
    wl = synth.workload("apdm512")
    offs = oracle.offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), wl.n, wl.obj_shape)
    st, nbytes = _dry(wl.n, wl.n_modes, wl.n_frames, wl.obj_shape, 0, offs)
    assert st == 0 and nbytes > 0


def test_subpixel_windows_match_oracle_bitwise():
    from paper_2008_11511_amd.plan import windows_from_positions
    rng = np.random.default_rng(3)
    pos = rng.uniform(-300.0, 300.0, (200000, 2))
    pos[:1000] = np.round(pos[:1000])                 # integer corners
    pos[1000:2000] = np.round(pos[1000:2000] * 4) / 4  # exact quarters
    got_o, got_f = windows_from_positions(pos, 256, (1024, 1200))
    want_o, want_f = oracle.windows_from_positions(pos, 256, (1024, 1200))
    np.testing.assert_array_equal(got_o, want_o)
    np.testing.assert_array_equal(got_f, want_f)
    h = _lib.lib()
    out_o = np.zeros((1, 2), np.int32)
    out_f = np.zeros((1, 2))
    bad = np.array([[-384.5, 0.0]])                    # corner -0.5
    assert h.ptycho_windows_from_positions(bad.ctypes.data, 1, 256, 1024, 1200, out_o.ctypes.data,
                                           out_f.ctypes.data) == -2
    assert not out_o.any() and not out_f.any()


def test_positions_plan_descriptor_and_arguments_are_checked():
    h = _lib.lib()
    sz = ctypes.c_size_t()
    d = _desc(flags=4)
    d.max_shift = 2.0
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(sz)) == 0
    d.max_shift = -1.0
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(sz)) == -1
    d.max_shift = float("nan")
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(sz)) == -1
    fake = ctypes.c_void_p(256)
    assert h.ptycho_plan_set_positions(None, fake, 1.0, 0.1) == -1
    assert h.ptycho_plan_positions(None, fake) == -1
    assert h.ptycho_refine_positions(None, fake, fake, fake, None) == -1


def test_automatic_stack_takes_up_to_32_gib_of_scratch():
    """The automatic stack is the largest whose scratch fits 32 GiB: a
    4000-frame scan of 512^2 frames with 4 modes (32 GiB of frame-modes) runs
    as one stack, a scan three times longer is split, and an explicit stack
    of 256 frames needs far less workspace."""
    h = _lib.lib()
    per = 4 * 512 * 512 * 8
    one = ctypes.c_size_t()
    d = _desc(n=512, n_modes=4, n_frames=4000, obj_ny=4096, obj_nx=4096)
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(one)) == 0
    assert one.value >= 4000 * per                 # the whole scan's scratch
    big = ctypes.c_size_t()
    d = _desc(n=512, n_modes=4, n_frames=12000, obj_ny=8192, obj_nx=8192)
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(big)) == 0
    assert (32 << 30) <= big.value < 12000 * per   # capped: several stacks
    small = ctypes.c_size_t()
    d = _desc(n=512, n_modes=4, n_frames=4000, obj_ny=4096, obj_nx=4096, stack=256)
    assert h.ptycho_workspace_bytes(ctypes.byref(d), ctypes.byref(small)) == 0
    assert 256 * per <= small.value < 1000 * per

"""Sub-pixel positions on the GPU (plans created with PTYCHO_FLAG_POSITIONS)
against the oracle's sub-pixel windows: every operator, the position shifts,
and AP and ML cycles that refine the positions on the device.  Positions are
float64 on both sides; the windows' fractions enter the GPU kernels in fp32."""
import sys

import numpy as np
import pytest

import oracle
import synth
from cases import make_problem, rel_l2, small

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

UPD = oracle.UPDATE_OBJECT | oracle.UPDATE_PROBE


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


def t_(a, dev, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)


def host(x):
    torch.cuda.synchronize()
    return x.cpu().numpy().astype(np.complex128 if x.is_complex() else np.float64)


def subpixel_problem(n=64, k=2, j=40, side=224, seed_offset=0, jitter=0.3):
    """Data taken at true sub-pixel positions; the start positions are off by
    +-jitter pixels; start object and probe near the truth."""
    wl = small("dm256", n=n, k=k, j=j, obj=(side, side), step=5.0, mask_frac=0.03, seed_offset=seed_offset)
    pb = make_problem(wl, start="ml")
    rng = np.random.default_rng(100 + seed_offset)
    pos_true = synth.spiral_positions(j, wl.step) + rng.uniform(-0.5, 0.5, (j, 2))
    offs_t, frac_t = oracle.windows_from_positions(pos_true, n, wl.obj_shape)
    inten = oracle.simulate_intensity(pb.obj_true, pb.probe_true, offs_t, frac=frac_t)
    iobs = synth.poisson_counts(inten, wl.seed)
    pos0 = pos_true + rng.choice([-jitter, jitter], size=(j, 2))
    return pb, pos_true, pos0, iobs


def make_positions_plan(pb, iobs, pos, dev, max_shift=2.0, mult=1.0, min_grad=0.1):
    from paper_2008_11511_amd import Plan
    mask = t_(pb.mask, dev, torch.uint8) if pb.mask is not None else None
    return Plan.with_positions(pos, t_(iobs, dev, torch.float32), mask, pb.wl.n_modes, pb.wl.obj_shape,
                               max_shift=max_shift, mult=mult, min_grad=min_grad)


def test_integer_positions_reproduce_the_integer_plan_bitwise(dev):
    from paper_2008_11511_amd import Plan
    pb = make_problem(small("dm256", n=64, k=2, j=30, obj=(192, 192), step=4.0, mask_frac=0.03), start="ml")
    say("positions plan with integer corners vs integer plan")
    wl = pb.wl
    # positions whose corners are exactly the integer offsets
    pos = pb.offsets.astype(np.float64) + wl.n / 2.0 - np.array(wl.obj_shape) / 2.0
    iobs = t_(pb.iobs, dev, torch.float32)
    mask = t_(pb.mask, dev, torch.uint8)
    a = Plan(pb.offsets, iobs, mask, wl.n_modes, wl.obj_shape)
    b = Plan.with_positions(pos, iobs, mask, wl.n_modes, wl.obj_shape, max_shift=1.0)
    out = []
    for plan in (a, b):
        o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
        psi = plan.psi_init(o, p)
        plan.dm_cycle(o, p, psi, 2, UPD)
        g_o, g_p, llk = plan.ml_grad(o, p)
        out.append([host(x) for x in (psi, o, p, g_o, g_p, llk)])
    for x, y in zip(*out):
        np.testing.assert_array_equal(x, y)


def test_subpixel_operators_match_oracle(dev):
    pb, pos_true, pos0, iobs = subpixel_problem()
    wl = pb.wl
    offs, frac = oracle.windows_from_positions(pos0, wl.n, wl.obj_shape)
    assert (frac > 0.05).any()
    say("sub-pixel operators vs oracle n=64 k=2 j=40")
    plan = make_positions_plan(pb, iobs, pos0, dev)
    np.testing.assert_array_equal(plan.offsets, offs)
    o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
    o0, p0 = pb.obj0, pb.probe0
    psi = plan.psi_init(o, p)
    assert rel_l2(host(psi), oracle.psi_init(o0, p0, offs, frac)) < 1e-6
    ic = plan.icalc(o, p)
    assert rel_l2(host(ic), oracle.simulate_intensity(o0, p0, offs, frac=frac)) < 1e-5
    llk = host(plan.llk(o, p))
    ref, nobs = oracle.llk(o0, p0, offs, iobs, pb.mask, frac=frac)
    assert llk[1] == nobs and abs(llk[0] - ref) < 1e-4 * abs(ref)
    g_o, g_p, _ = plan.ml_grad(o, p)
    r_o, r_p, _ = oracle.ml_grad(o0, p0, offs, iobs, pb.mask, frac=frac)
    assert rel_l2(host(g_o), r_o) < 1e-4 and rel_l2(host(g_p), r_p) < 1e-4
    rng = np.random.default_rng(5)
    d_o = (rng.standard_normal(o0.shape) + 1j * rng.standard_normal(o0.shape)) * 1e-2
    d_p = (rng.standard_normal(p0.shape) + 1j * rng.standard_normal(p0.shape)) * 1e-2
    c = host(plan.ml_linesearch(o, p, t_(d_o, dev, torch.complex64), t_(d_p, dev, torch.complex64)))
    l1, l2 = oracle.linesearch_coefs(o0, p0, d_o.astype(np.complex64), d_p.astype(np.complex64), offs, iobs,
                                     pb.mask, frac=frac)
    assert abs(c[0] - l1) < 1e-4 * abs(l1) and abs(c[1] - l2) < 1e-4 * abs(l2)
    # one AP and one DM cycle
    o_ap, p_ap = o.clone(), p.clone()
    plan.ap_cycle(o_ap, p_ap, 1, UPD)
    ro, rp = oracle.ap_cycle(o0, p0, offs, iobs, pb.mask, UPD, frac=frac)
    assert rel_l2(host(o_ap), ro) < 1e-4 and rel_l2(host(p_ap), rp) < 1e-4
    plan.dm_cycle(o, p, psi, 1, UPD)
    ro, rp, rpsi = oracle.dm_cycle(o0, p0, oracle.psi_init(o0, p0, offs, frac), offs, iobs, pb.mask, UPD, frac=frac)
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4 and rel_l2(host(psi), rpsi) < 1e-4


def test_subpixel_position_shifts_match_oracle(dev):
    pb, pos_true, pos0, iobs = subpixel_problem(seed_offset=1)
    wl = pb.wl
    offs, frac = oracle.windows_from_positions(pos0, wl.n, wl.obj_shape)
    say("sub-pixel position shifts vs oracle")
    psi = oracle.fourier_project(oracle.exit_waves(pb.obj0, pb.probe0, offs, frac), iobs, pb.mask)
    psi64 = psi.astype(np.complex64)
    ref, e_ref = oracle.position_shifts(pb.obj0, pb.probe0, psi64.astype(np.complex128), offs, frac)
    plan = make_positions_plan(pb, iobs, pos0, dev)
    got = host(plan.position_shifts(t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64),
                                    t_(psi64, dev, torch.complex64)))
    scale = np.abs(ref).max()
    assert scale > 0.02
    assert np.abs(got[:, :2] - ref).max() <= 1e-4 * scale
    np.testing.assert_allclose(got[:, 2], e_ref, rtol=1e-5)


def _oracle_ap_refinement(pb, iobs, pos0, cycles, mult=1.0, max_shift=2.0, min_grad=0.1):
    o, p, pos = pb.obj0, pb.probe0, pos0.copy()
    for _ in range(cycles):
        offs, frac = oracle.windows_from_positions(pos, pb.wl.n, pb.wl.obj_shape)
        psi = oracle.fourier_project(oracle.exit_waves(o, p, offs, frac), iobs, pb.mask)
        o, p = oracle.overlap_update(o, p, psi, offs, UPD, frac=frac)
        sh, e = oracle.position_shifts(o, p, psi, offs, frac)
        pos = oracle.update_positions(pos, pos0, sh, e, mult, max_shift, min_grad)
    return o, p, pos


def test_ap_cycles_with_position_updates_follow_oracle(dev):
    from paper_2008_11511_amd import UPDATE_POSITIONS
    pb, pos_true, pos0, iobs = subpixel_problem(seed_offset=2)
    say("3 AP cycles with position updates vs oracle")
    ro, rp, rpos = _oracle_ap_refinement(pb, iobs, pos0, 3)
    plan = make_positions_plan(pb, iobs, pos0, dev)
    o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
    plan.ap_cycle(o, p, 3, UPD | UPDATE_POSITIONS)
    gpos = host(plan.positions())
    assert np.abs(gpos - pos0).max() > 0.05                   # the positions moved
    assert np.abs(gpos - rpos).max() < 1e-3
    assert rel_l2(host(o), ro) < 1e-3 and rel_l2(host(p), rp) < 1e-3


def test_ml_cycles_with_position_updates_follow_oracle(dev):
    from paper_2008_11511_amd import UPDATE_POSITIONS
    pb, pos_true, pos0, iobs = subpixel_problem(seed_offset=3)
    say("3 CG cycles with position updates vs oracle")
    o_r, p_r, pos, st = pb.obj0, pb.probe0, pos0.copy(), oracle.CGState()
    for _ in range(3):
        offs, frac = oracle.windows_from_positions(pos, pb.wl.n, pb.wl.obj_shape)
        sh, e = oracle.ml_position_shifts(o_r, p_r, offs, iobs, pb.mask, frac=frac)
        o_r, p_r = oracle.ml_cycle(o_r, p_r, st, offs, iobs, pb.mask, update=UPD, frac=frac)
        pos = oracle.update_positions(pos, pos0, sh, e)
    plan = make_positions_plan(pb, iobs, pos0, dev)
    o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
    state = plan.ml_state()
    hist = torch.zeros(3, dtype=torch.float64, device=dev)
    plan.ml_cycle(o, p, state, 3, UPD | UPDATE_POSITIONS, reset=True, hist=hist)
    gpos = host(plan.positions())
    assert np.abs(gpos - pos0).max() > 0.02
    assert np.abs(gpos - pos).max() < 1e-3
    np.testing.assert_allclose(host(hist), st.history, rtol=1e-4)
    assert rel_l2(host(o), o_r) < 1e-3 and rel_l2(host(p), p_r) < 1e-3


def test_positions_stay_within_max_shift_and_the_object(dev):
    from paper_2008_11511_amd import UPDATE_POSITIONS
    pb, pos_true, pos0, iobs = subpixel_problem(seed_offset=4, jitter=0.6)
    say("10 AP cycles with aggressive position steps stay within max_shift")
    plan = make_positions_plan(pb, iobs, pos0, dev, max_shift=0.75, mult=4.0, min_grad=0.0)
    o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
    plan.ap_cycle(o, p, 10, UPD | UPDATE_POSITIONS)
    gpos = host(plan.positions())
    assert np.abs(gpos - pos0).max() <= 0.75 + 1e-12
    assert np.isclose(np.abs(gpos - pos0).max(), 0.75)       # the bound is reached and holds
    oracle.windows_from_positions(gpos, pb.wl.n, pb.wl.obj_shape)     # inside the object
    assert np.isfinite(host(o)).all()


def test_position_shifts_refuse_misaligned_arrays_before_any_work(dev):
    """The shift kernel reads two pixels in one 16-byte load: exit waves or a
    probe that are only 8-byte aligned are refused by the host checks."""
    from paper_2008_11511_amd import PtychoError
    pb, pos_true, pos0, iobs = subpixel_problem(seed_offset=5)
    wl = pb.wl
    say("misaligned exit waves and probe are refused")
    plan = make_positions_plan(pb, iobs, pos0, dev)
    o, p = t_(pb.obj0, dev, torch.complex64), t_(pb.probe0, dev, torch.complex64)
    shape = (wl.n_frames, wl.n_modes, wl.n, wl.n)
    n_psi = int(np.prod(shape))
    big = torch.zeros(n_psi + 1, dtype=torch.complex64, device=dev)
    psi_bad = big[1:].view(shape)
    assert psi_bad.data_ptr() % 16 == 8
    pos_before = host(plan.positions())
    with pytest.raises(PtychoError) as e:
        plan.position_shifts(o, p, psi_bad)
    assert e.value.code == -1
    with pytest.raises(PtychoError):
        plan.refine(o, p, psi_bad)
    pbig = torch.zeros(p.numel() + 1, dtype=torch.complex64, device=dev)
    p_bad = pbig[1:].view(p.shape)
    p_bad.copy_(p)
    psi_ok = torch.zeros(shape, dtype=torch.complex64, device=dev)
    with pytest.raises(PtychoError):
        plan.position_shifts(o, p_bad, psi_ok)
    np.testing.assert_array_equal(host(plan.positions()), pos_before)     # nothing moved
    # aligned arrays work
    out = host(plan.position_shifts(o, p, psi_ok))
    assert np.isfinite(out).all()


@pytest.mark.parametrize("n", [8, 16, 32, 128, 512, 1024, 2048])
def test_position_shifts_match_oracle_at_every_size(dev, n):
    """The shift kernel's thread layout changes with N (pairs of columns per
    thread, row groups below 512 points, several pairs per thread from 1024):
    integer and sub-pixel windows against the oracle at every supported size,
    random object, probe and exit waves, windows near the object's border."""
    from paper_2008_11511_amd import Plan
    rng = np.random.default_rng(1000 + n)
    k = 1 if n == 2048 else 2
    j = 3
    side = n + 24
    say(f"position shifts at n={n}, {j} frames, {k} modes")
    obj = (rng.standard_normal((side, side)) + 1j * rng.standard_normal((side, side))).astype(np.complex64)
    probe = (rng.standard_normal((k, n, n)) + 1j * rng.standard_normal((k, n, n))).astype(np.complex64)
    psi = (rng.standard_normal((j, k, n, n)) + 1j * rng.standard_normal((j, k, n, n))).astype(np.complex64)
    # corners: one near each border (sub-pixel plans need max_shift + 1 pixels of margin)
    t = np.array([[2.25, 3.5], [side - n - 2.75, 7.125], [11.5, side - n - 2.5]])
    pos = t - side / 2.0 + n / 2.0
    offs, frac = oracle.windows_from_positions(pos, n, (side, side))
    iobs = torch.zeros((j, n, n), dtype=torch.float32, device=dev)
    o_d, p_d, psi_d = t_(obj, dev, torch.complex64), t_(probe, dev, torch.complex64), t_(psi, dev, torch.complex64)
    for sub in (False, True):
        if sub:
            plan = Plan.with_positions(pos, iobs, None, k, (side, side), max_shift=1.0)
            ref, e_ref = oracle.position_shifts(obj, probe, psi, offs, frac)
        else:
            plan = Plan(offs, iobs, None, k, (side, side))
            ref, e_ref = oracle.position_shifts(obj, probe, psi, offs)
        got = host(plan.position_shifts(o_d, p_d, psi_d))
        scale = max(np.abs(ref).max(), 1e-3)
        assert np.abs(got[:, :2] - ref).max() <= 1e-3 * scale, (n, sub)
        np.testing.assert_allclose(got[:, 2], e_ref, rtol=1e-4)
        plan.close()

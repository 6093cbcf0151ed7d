"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative L2 <= 1e-4 after one cycle / one gradient, <= 1e-3 on
the object after many cycles; integer work (offsets, window extraction, the
mask decision) bit-exact.  Every case prints its name before touching the GPU.
"""
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
    P.lib()        # raises if the HIP library is missing: no fallback
    return torch.device("cuda:0")


def to_dev(a, dev, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)


def make_plan(pb, dev, stack=0):
    from paper_2008_11511_amd import Plan
    iobs = to_dev(pb.iobs, dev, torch.float32)
    mask = to_dev(pb.mask, dev, torch.uint8) if pb.mask is not None else None
    return Plan(pb.offsets, iobs, mask, pb.wl.n_modes, pb.wl.obj_shape, stack=stack)


def state(pb, dev):
    return (to_dev(pb.obj0, dev, torch.complex64).contiguous(),
            to_dev(pb.probe0, dev, torch.complex64).contiguous())


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


# ---------------------------------------------------------------- FFT -----
@pytest.mark.parametrize("n", [8, 16, 32, 64, 128, 256, 512, 1024, 2048])
def test_fft2_matches_oracle(dev, n):
    from paper_2008_11511_amd import fft2
    rng = np.random.default_rng(n)
    count = 3
    x = (rng.standard_normal((count, n, n)) + 1j * rng.standard_normal((count, n, n))).astype(np.complex64)
    say(f"fft2 n={n} count={count}")
    xd = to_dev(x, dev, torch.complex64)
    f = host(fft2(xd))
    b = host(fft2(xd, inverse=True))
    assert rel_l2(f, oracle.fft2(x)) < 2e-6
    assert rel_l2(b, oracle.ifft2(x)) < 2e-6
    rt = host(fft2(fft2(xd), inverse=True))
    assert rel_l2(rt, x) < 2e-6
    np.testing.assert_allclose((abs(f) ** 2).sum(axis=(1, 2)), (abs(x.astype(np.complex128)) ** 2).sum(axis=(1, 2)),
                               rtol=1e-5)


# ------------------------------------------------------ exact extraction --
def test_views_are_bit_exact(dev):
    wl = small("dm256", n=64, k=2, j=37, obj=(300, 280), step=8.0)
    offs = oracle.offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), wl.n, wl.obj_shape)
    ny, nx = wl.obj_shape
    obj = np.arange(ny * nx, dtype=np.float64).reshape(ny, nx).astype(np.complex64)   # exact in fp32
    probe = np.ones((2, 64, 64), np.complex64)
    probe[1] *= 1j
    from paper_2008_11511_amd import Plan
    say("psi_init bit-exact views")
    iobs = torch.zeros((wl.n_frames, 64, 64), dtype=torch.float32, device=dev)
    plan = Plan(offs, iobs, None, 2, wl.obj_shape)
    psi = host(plan.psi_init(to_dev(obj, dev, torch.complex64), to_dev(probe, dev, torch.complex64)))
    exp = oracle.exit_waves(obj, probe, offs)
    assert np.array_equal(psi, exp)
    # the offsets the plan was built from are the oracle's, bit for bit
    from paper_2008_11511_amd import offsets_from_positions
    np.testing.assert_array_equal(offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), 64,
                                                         wl.obj_shape), offs)


# ------------------------------------------------- forward model / LLK ----
@pytest.mark.parametrize("n,k,j", [(8, 2, 25), (16, 1, 37), (32, 2, 7), (64, 1, 100), (128, 3, 21), (256, 3, 12),
                                   (512, 4, 5), (1024, 2, 3), (2048, 1, 2)])
def test_icalc_and_llk_match_oracle(dev, n, k, j):
    side = max(256, 2 * n + 64)
    wl = small("dm256", n=n, k=k, j=j, obj=(side, side), step=max(2.0, n / 16), mask_frac=0.03 if n >= 64 else 0)
    pb = make_problem(wl, start="ml")
    say(f"icalc/llk n={n} k={k} j={j}")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    ic_ref = oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets)
    assert rel_l2(ic, ic_ref) < 1e-5
    for model in oracle.LLK_MODELS:
        llk = host(plan.llk(o, p, model=model))
        ref, nobs = oracle.llk(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, model=model)
        assert llk[1] == nobs
        assert abs(llk[0] - ref) <= 1e-4 * abs(ref), model


def test_noise_model_llk_near_the_fit_and_unknown_model(dev):
    """Near a perfect fit the three models agree to second order; fp32 terms
    must keep that (the Euclidean one takes a difference of square roots)."""
    wl = small("dm256", n=64, k=2, j=30, obj=(256, 256), step=4.0, mask_frac=0.03)
    pb = make_problem(wl, start="truth", noiseless=True)
    say("llk near the fit, all models")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    # a 1e-3 probe scale: I = Iobs (1 + d), d ~ 2e-3
    p = p * (1.0 + 1e-3)
    pp = pb.probe0 * (1.0 + 1e-3)
    vals = {}
    for model in oracle.LLK_MODELS:
        llk = host(plan.llk(o, p, model=model))
        ref, _ = oracle.llk(pb.obj0, pp.astype(np.complex64).astype(np.complex128), pb.offsets, pb.iobs,
                            pb.mask, model=model)
        assert abs(llk[0] - ref) <= 2e-3 * abs(ref), model
        vals[model] = llk[0]
    assert abs(vals["gaussian"] / vals["poisson"] - 1) < 0.05
    assert abs(vals["euclidean"] / vals["poisson"] - 1) < 0.05
    from paper_2008_11511_amd._lib import lib
    from paper_2008_11511_amd.plan import _ptr
    out = torch.empty(2, dtype=torch.float64, device=dev)
    assert lib().ptycho_llk_model(plan._h, _ptr(o), _ptr(p), 7, _ptr(out)) == -1
    with pytest.raises(ValueError):
        plan.llk(o, p, model="cauchy")


# ------------------------------------------------------------- AP / DM ----
# Cycle parity is taken from a start near the truth (smooth 0.2 rad object
# phase error, 10% probe amplitude error).  From the benchmark start O = 1
# the exit waves' far field is below fp32 resolution on most pixels while
# Iobs is not, so the modulus projection assigns those pixels the phase of
# rounding noise: the oracle itself moves by percents under 6e-8 input noise
# there (tests/test_oracle_conditioning.py).  What is unique from that start,
# the projected modulus, is checked separately below.
def test_ap_one_cycle_full_ap64(dev):
    pb = make_problem(synth.workload("ap64"), start="ml")
    say("AP one cycle, 64x64, 1 mode, 100 frames")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    plan.ap_cycle(o, p, 1, UPD)
    ro, rp = oracle.ap_cycle(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, UPD)
    assert rel_l2(host(o), ro) < 1e-4
    assert rel_l2(host(p), rp) < 1e-4


def test_ap_ten_cycles_full_ap64(dev):
    pb = make_problem(synth.workload("ap64"), start="ml")
    say("AP ten cycles, 64x64")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    plan.ap_cycle(o, p, 10, UPD)
    ro, rp = pb.obj0, pb.probe0
    for _ in range(10):
        ro, rp = oracle.ap_cycle(ro, rp, pb.offsets, pb.iobs, pb.mask, UPD)
    assert rel_l2(host(o), ro) < 1e-3
    assert rel_l2(host(p), rp) < 1e-3


@pytest.mark.parametrize("n,k,j,stack", [(64, 3, 60, 0), (128, 3, 33, 7), (256, 3, 24, 0), (512, 4, 6, 4),
                                         (16, 2, 37, 5), (32, 1, 9, 3), (8, 3, 30, 4), (1024, 4, 3, 2),
                                         (2048, 2, 2, 0)])
def test_dm_one_cycle(dev, n, k, j, stack):
    side = max(256, 2 * n + 64)
    wl = small("dm256", n=n, k=k, j=j, obj=(side, side), step=max(2.0, n / 16), mask_frac=0.03 if n >= 64 else 0)
    pb = make_problem(wl, start="ml")
    say(f"DM one cycle n={n} k={k} j={j} stack={stack}")
    plan = make_plan(pb, dev, stack=stack)
    o, p = state(pb, dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, UPD)
    assert rel_l2(host(psi), rpsi) < 1e-4
    assert rel_l2(host(o), ro) < 1e-4
    assert rel_l2(host(p), rp) < 1e-4


def test_dm_many_cycles(dev):
    wl = small("dm256", n=64, k=2, j=80, obj=(256, 256), step=6.0, mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    say("DM 50 cycles n=64 k=2 j=80")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 50, UPD)
    ro, rp = pb.obj0, pb.probe0
    rpsi = oracle.psi_init(ro, rp, pb.offsets)
    for _ in range(50):
        ro, rp, rpsi = oracle.dm_cycle(ro, rp, rpsi, pb.offsets, pb.iobs, pb.mask, UPD)
    assert rel_l2(host(o), ro) < 1e-3
    assert rel_l2(host(p), rp) < 1e-3


def test_update_flags(dev):
    wl = small("dm256", n=64, k=2, j=30, obj=(200, 200), step=5.0, mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    for upd in (oracle.UPDATE_OBJECT, oracle.UPDATE_PROBE, 0):
        say(f"AP update flag {upd}")
        plan = make_plan(pb, dev)
        o, p = state(pb, dev)
        plan.ap_cycle(o, p, 1, upd)
        ro, rp = oracle.ap_cycle(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, upd)
        assert rel_l2(host(o), ro) < 1e-4
        assert rel_l2(host(p), rp) < 1e-4


@pytest.mark.parametrize("n,k", [(64, 1), (256, 1)])
def test_projection_modulus_from_benchmark_start(dev, n, k):
    """From O = 1 the phases of weak pixels are not defined in fp32, but the
    projected intensity is: |F Psi1|^2 = Iobs at every good pixel after the
    first DM cycle (Psi1 = P_F(Phi0)), and bad pixels keep |F Phi0|^2."""
    side = max(256, 2 * n + 64)
    wl = small("dm256", n=n, k=k, j=12, obj=(side, side), step=n / 16, mask_frac=0.03)
    pb = make_problem(wl)
    say(f"projected modulus n={n}")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    psi0 = plan.psi_init(o, p)
    psi = psi0.clone()
    plan.dm_cycle(o, p, psi, 1, 0)
    from paper_2008_11511_amd import fft2
    f1 = host(fft2(psi.view(-1, n, n))).reshape(pb.wl.n_frames, k, n, n)
    f0 = host(fft2(psi0.view(-1, n, n))).reshape(pb.wl.n_frames, k, n, n)
    i1 = (abs(f1) ** 2).sum(axis=1)
    i0 = (abs(f0) ** 2).sum(axis=1)
    good = pb.mask == 0
    tot = pb.iobs.sum()
    assert np.abs(i1[:, good] - pb.iobs[:, good]).sum() < 1e-4 * tot
    assert np.abs(i1[:, ~good] - i0[:, ~good]).sum() < 1e-4 * i0.sum()


# ---------------------------------------------------- mask / determinism ---
def test_mask_is_bit_exact_and_outputs_reproducible(dev):
    wl = small("dm256", n=128, k=3, j=20, obj=(320, 320), step=8.0, mask_frac=0.05)
    pb = make_problem(wl)
    assert pb.mask is not None and pb.mask.any()
    iobs2 = pb.iobs.copy()
    iobs2[:, pb.mask != 0] = 12345.0           # garbage under the mask
    pb2 = make_problem(wl)
    pb2.iobs = iobs2
    outs = []
    for q in (pb, pb, pb2):
        say("DM 2 cycles, mask garbage / repeat")
        plan = make_plan(q, dev)
        o, p = state(q, dev)
        psi = plan.psi_init(o, p)
        plan.dm_cycle(o, p, psi, 2, UPD)
        llk = plan.llk(o, p)
        outs.append((host(o), host(p), host(psi), host(llk)))
    for a, b in zip(outs[0], outs[1]):
        assert np.array_equal(a, b)            # run to run: bitwise
    for a, b in zip(outs[0], outs[2]):
        assert np.array_equal(a, b)            # masked pixels never read


def test_stack_size_does_not_change_the_result(dev):
    wl = small("dm256", n=64, k=2, j=50, obj=(256, 256), step=6.0, mask_frac=0.03)
    pb = make_problem(wl)
    res = []
    for st in (1, 7, 0):
        say(f"AP stack={st}")
        plan = make_plan(pb, dev, stack=st)
        o, p = state(pb, dev)
        plan.ap_cycle(o, p, 2, UPD)
        res.append((host(o), host(p)))
    for o, p in res[1:]:
        assert rel_l2(o, res[0][0]) < 1e-6
        assert rel_l2(p, res[0][1]) < 1e-6


# ----------------------------------------------------------------- ML -----
@pytest.mark.parametrize("n,k,j", [(64, 1, 40), (256, 3, 16)])
def test_ml_grad_and_linesearch_match_oracle(dev, n, k, j):
    side = max(256, 2 * n + 64)
    wl = small("ml256", n=n, k=k, j=j, obj=(side, side), step=max(2.0, n / 16), mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    say(f"ML grad n={n} k={k} j={j}")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    go, gp, llk = plan.ml_grad(o, p)
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask)
    assert rel_l2(host(go), ro) < 1e-4
    assert rel_l2(host(gp), rp) < 1e-4
    assert abs(host(llk)[0] - rl) < 1e-4 * abs(rl)
    rng = np.random.default_rng(5)
    d_o = (rng.standard_normal(pb.obj0.shape) + 1j * rng.standard_normal(pb.obj0.shape)).astype(np.complex64) * 1e-2
    d_p = (rng.standard_normal(pb.probe0.shape) + 1j * rng.standard_normal(pb.probe0.shape)).astype(np.complex64)
    d_p *= 1e-2 * np.abs(pb.probe0).max()
    say(f"ML line search n={n}")
    coef = host(plan.ml_linesearch(o, p, to_dev(d_o, dev, torch.complex64), to_dev(d_p, dev, torch.complex64)))
    r1, r2 = oracle.linesearch_coefs(pb.obj0, pb.probe0, d_o, d_p, pb.offsets, pb.iobs, pb.mask)
    assert abs(coef[0] - r1) <= 1e-4 * abs(r1)
    assert abs(coef[1] - r2) <= 1e-4 * abs(r2)


def test_ml_cycles_match_oracle(dev):
    wl = small("ml256", n=64, k=2, j=40, obj=(256, 256), step=5.0, mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    upd = UPD
    say("ML 5 cycles n=64 k=2")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    st = plan.ml_state()
    hist = torch.zeros(5, dtype=torch.float64, device=dev)
    plan.ml_cycle(o, p, st, 5, upd, reset=True, hist=hist)
    cg = oracle.CGState()
    ro, rp = pb.obj0, pb.probe0
    for _ in range(5):
        ro, rp = oracle.ml_cycle(ro, rp, cg, pb.offsets, pb.iobs, pb.mask, update=upd)
    h = host(hist)
    np.testing.assert_allclose(h, cg.history, rtol=1e-4)
    assert rel_l2(host(o), ro) < 1e-3
    assert rel_l2(host(p), rp) < 1e-3


# ------------------------------------------------------------ autograd ----
def test_poisson_llk_autograd_matches_finite_differences_and_oracle(dev):
    """torch.autograd over the hand-written adjoint: gradients against central
    finite differences (h = 1e-3 of the RMS value) of the FP64 oracle LLK at
    20 object and 20 probe pixels whose gradient exceeds a tenth of the
    largest, each within 1% of its difference, and against the full oracle
    gradient."""
    import paper_2008_11511_amd as P
    wl = small("ml256", n=64, k=2, j=30, obj=(192, 192), step=4.0, mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    say("autograd PoissonLLK")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    o.requires_grad_(True)
    p.requires_grad_(True)
    loss = P.poisson_llk(o, p, plan)
    loss.backward()
    go, gp = host(o.grad), host(p.grad)
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask)
    assert abs(float(loss.detach().cpu()) - rl) < 1e-4 * abs(rl)
    assert rel_l2(go, ro) < 1e-4 and rel_l2(gp, rp) < 1e-4
    # torch's own convention check: d|z|^2 = 2z
    z = torch.tensor([1.0 + 2.0j], dtype=torch.complex64, requires_grad=True)
    (z.abs() ** 2).sum().backward()
    assert torch.allclose(z.grad, 2 * z.detach())
    rng = np.random.default_rng(7)
    f_o = lambda x: oracle.llk(x, pb.probe0, pb.offsets, pb.iobs, pb.mask)[0]
    f_p = lambda x: oracle.llk(pb.obj0, x, pb.offsets, pb.iobs, pb.mask)[0]
    for x0, g, f in ((pb.obj0, go, f_o), (pb.probe0, gp, f_p)):
        h = 1e-3 * np.sqrt((abs(x0) ** 2).mean())
        cand = np.flatnonzero(abs(g) > 0.1 * abs(g).max())
        for i in rng.choice(cand, 20, replace=False):
            e = np.zeros(x0.shape, complex)
            e.flat[i] = h
            fd = complex((f(x0 + e) - f(x0 - e)) / (2 * h), (f(x0 + 1j * e) - f(x0 - 1j * e)) / (2 * h))
            assert abs(g.flat[i] - fd) <= 1e-2 * abs(fd) + 1e-6 * abs(g).max(), (i, g.flat[i], fd)


# ---------------------------------------------------------- background ----
def _bg_problem(n=64, k=2, j=50, bg_level=5.0, start="ml"):
    side = max(256, 2 * n + 64)
    wl = small("dm256", n=n, k=k, j=j, obj=(side, side), step=max(2.0, n / 16), mask_frac=0.03)
    return make_problem(wl, start=start, bg_level=bg_level)


@pytest.mark.parametrize("n,k", [(64, 2), (256, 3)])
def test_background_in_every_operator_matches_oracle(dev, n, k):
    pb = _bg_problem(n, k, j=40 if n == 64 else 12)
    say(f"background: icalc/llk/grad/dm n={n} k={k}")
    plan = make_plan(pb, dev)
    bg = to_dev(pb.bg0, dev, torch.float32)
    plan.set_background(bg)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    assert rel_l2(ic, oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets, bg=pb.bg0)) < 1e-5
    for model in oracle.LLK_MODELS:
        llk = host(plan.llk(o, p, model=model))
        ref, _ = oracle.llk(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, model=model, bg=pb.bg0)
        assert abs(llk[0] - ref) <= 1e-4 * abs(ref), model
    go, gp, _ = plan.ml_grad(o, p)
    ro, rp, _ = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, bg=pb.bg0)
    assert rel_l2(host(go), ro) < 1e-4 and rel_l2(host(gp), rp) < 1e-4
    d_o, d_p = (pb.obj0 * 0.01j).astype(np.complex64), (pb.probe0 * 0.02).astype(np.complex64)
    c = host(plan.ml_linesearch(o, p, to_dev(d_o, dev, torch.complex64), to_dev(d_p, dev, torch.complex64)))
    l1, l2 = oracle.linesearch_coefs(pb.obj0, pb.probe0, d_o.astype(np.complex128), d_p.astype(np.complex128),
                                     pb.offsets, pb.iobs, pb.mask, bg=pb.bg0)
    assert abs(c[0] - l1) <= 1e-4 * abs(l1) and abs(c[1] - l2) <= 1e-4 * abs(l2)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, bg=pb.bg0)
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4 and rel_l2(host(psi), rpsi) < 1e-4
    # the background is only read
    assert np.array_equal(host(bg), pb.bg0)


@pytest.mark.parametrize("n,k,stack,cycles,start", [(64, 2, 0, 1, "ml"), (64, 1, 7, 1, "ml"), (128, 3, 0, 5, "ml"),
                                                    (64, 2, 0, 3, "truth")])
def test_ap_background_refinement_matches_oracle(dev, n, k, stack, cycles, start):
    from paper_2008_11511_amd import Plan, UPDATE_BACKGROUND
    pb = _bg_problem(n, k, j=45 if n == 64 else 30, bg_level=5.0 if start == "ml" else 100.0, start=start)
    say(f"AP background refinement n={n} k={k} stack={stack} cycles={cycles} start={start}")
    iobs = to_dev(pb.iobs, dev, torch.float32)
    mask = to_dev(pb.mask, dev, torch.uint8)
    plan = Plan(pb.offsets, iobs, mask, k, pb.wl.obj_shape, stack=stack, background_update=True)
    bg = to_dev(pb.bg0, dev, torch.float32)
    plan.set_background(bg)
    o, p = state(pb, dev)
    plan.ap_cycle(o, p, cycles, UPD | UPDATE_BACKGROUND)
    ro, rp, rb = pb.obj0, pb.probe0, pb.bg0
    for _ in range(cycles):
        ro, rp, rb = oracle.ap_cycle(ro, rp, pb.offsets, pb.iobs, pb.mask, UPD | oracle.UPDATE_BACKGROUND, bg=rb)
    tol = 1e-4 if cycles == 1 else 1e-3
    assert rel_l2(host(bg), rb) < tol
    assert rel_l2(host(o), ro) < tol and rel_l2(host(p), rp) < tol
    if start == "truth":
        # from the true object and probe the refinement moves the background
        # (30% low at the start) towards the truth
        assert rel_l2(host(bg), pb.bg_true) < rel_l2(pb.bg0, pb.bg_true) - 0.01


def test_background_update_arguments_are_checked(dev):
    from paper_2008_11511_amd import Plan, PtychoError, UPDATE_BACKGROUND
    pb = _bg_problem(64, 1, j=10)
    say("background argument checks")
    iobs = to_dev(pb.iobs, dev, torch.float32)
    o, p = state(pb, dev)
    plain = Plan(pb.offsets, iobs, None, 1, pb.wl.obj_shape)
    plain.set_background(to_dev(pb.bg0, dev, torch.float32))
    with pytest.raises(PtychoError):           # no workspace for the refinement
        plain.ap_cycle(o, p, 1, UPD | UPDATE_BACKGROUND)
    flagged = Plan(pb.offsets, iobs, None, 1, pb.wl.obj_shape, background_update=True)
    with pytest.raises(PtychoError):           # no background set
        flagged.ap_cycle(o, p, 1, UPD | UPDATE_BACKGROUND)
    flagged.set_background(to_dev(pb.bg0, dev, torch.float32))
    psi = flagged.psi_init(o, p)
    with pytest.raises(PtychoError):           # DM does not refine the background
        flagged.dm_cycle(o, p, psi, 1, UPD | UPDATE_BACKGROUND)
    with pytest.raises(ValueError):
        flagged.set_background(torch.zeros((32, 32), dtype=torch.float32, device=dev))


# ------------------------------------------------ position refinement ----
def test_position_shifts_match_oracle(dev):
    from paper_2008_11511_amd import Plan
    wl = small("dm256", n=64, k=2, j=30, obj=(256, 256), step=5.0, mask_frac=0.03)
    pb = make_problem(wl, start="ml")
    # two more frames on the object's corners: one-sided gradients there
    offs = np.concatenate([pb.offsets, [[0, 0], [256 - 64, 256 - 64]]]).astype(np.int32)
    say("position shifts vs oracle, 32 frames incl. corners")
    o64 = pb.obj0.astype(np.complex64)
    p64 = pb.probe0.astype(np.complex64)
    # exit waves from the oracle's projection of perturbed views
    psi = oracle.fourier_project(oracle.exit_waves(pb.obj_true, pb.probe_true, offs) * 1.02,
                                 oracle.simulate_intensity(pb.obj_true, pb.probe_true, offs), pb.mask)
    psi64 = psi.astype(np.complex64)
    ref, e_ref = oracle.position_shifts(o64.astype(np.complex128), p64.astype(np.complex128),
                                        psi64.astype(np.complex128), offs)
    iobs = torch.zeros((len(offs), 64, 64), dtype=torch.float32, device=dev)
    plan = Plan(offs, iobs, None, 2, wl.obj_shape)
    got = host(plan.position_shifts(to_dev(o64, dev, torch.complex64), to_dev(p64, dev, torch.complex64),
                                    to_dev(psi64, dev, torch.complex64)))
    scale = np.abs(ref).max()
    assert scale > 0.05
    assert np.abs(got[:, :2] - ref).max() <= 1e-4 * scale
    np.testing.assert_allclose(got[:, 2], e_ref, rtol=1e-5)


def test_position_update_matches_oracle_bitwise(dev):
    """ptycho_update_positions against the oracle's update rule: odd and even
    frame counts, tied energies, filtered frames, clipping on both sides."""
    from paper_2008_11511_amd.plan import update_positions
    rng = np.random.default_rng(8)
    for j, mult, mx, mg in ((201, 1.0, 2.0, 0.1), (200, 0.5, 1.0, 0.5), (7, 2.0, 3.0, 0.0), (1, 1.0, 2.0, 0.1),
                            (4096, 1.3, 0.75, 0.8)):
        say(f"position update: {j} frames, mult {mult}, max_shift {mx}, min_grad {mg}")
        pos0 = rng.uniform(-50, 50, (j, 2))
        pos = pos0 + rng.uniform(-2.5, 2.5, (j, 2))
        shifts = np.concatenate([rng.normal(0, 0.7, (j, 2)), rng.lognormal(0, 1.5, (j, 1))], axis=1)
        shifts[: j // 4, 2] = shifts[0, 2]             # ties in the energies
        want = oracle.update_positions(pos, pos0, shifts[:, :2], shifts[:, 2], mult, mx, mg)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        got = update_positions(t(pos), t(pos0), t(shifts), mult, mx, mg).cpu().numpy()
        np.testing.assert_array_equal(got, want)
        # in place
        pos_d = t(pos)
        update_positions(pos_d, t(pos0), t(shifts), mult, mx, mg, out=pos_d)
        np.testing.assert_array_equal(pos_d.cpu().numpy(), want)


def test_position_refinement_follows_oracle(dev):
    from paper_2008_11511_amd import Plan
    from paper_2008_11511_amd.plan import refine_positions
    wl = small("dm256", n=64, k=1, j=60, obj=(256, 256), step=5.0, mask_frac=0.0)
    pb = make_problem(wl, start="truth")
    pos_true = synth.spiral_positions(wl.n_frames, wl.step)
    off_true = oracle.offsets_from_positions(pos_true, wl.n, wl.obj_shape)
    rng = np.random.default_rng(1)
    err = np.zeros_like(pos_true)
    sel = rng.random(len(pos_true)) < 0.4
    err[sel] = rng.choice([-0.4, 0.4], size=(sel.sum(), 2))
    pos0 = pos_true + err
    say("position refinement: 2 AP cycles with position updates")
    # oracle
    pos, o, p = pos0.copy(), pb.obj0, pb.probe0
    for _ in range(2):
        offs = oracle.offsets_from_positions(pos, wl.n, wl.obj_shape)
        psi = oracle.fourier_project(oracle.exit_waves(o, p, offs), pb.iobs, pb.mask)
        o, p = oracle.overlap_update(o, p, psi, offs, UPD)
        sh, e = oracle.position_shifts(o, p, psi, offs)
        pos = oracle.update_positions(pos, pos0, sh, e)
    # GPU
    gpos = pos0.copy()
    plan = Plan(oracle.offsets_from_positions(gpos, wl.n, wl.obj_shape), to_dev(pb.iobs, dev, torch.float32), None,
                1, wl.obj_shape)
    go, gp = state(pb, dev)
    psi_d = torch.empty((wl.n_frames, 1, 64, 64), dtype=torch.complex64, device=dev)
    start_off = plan.offsets.copy()
    for _ in range(2):
        plan.ap_cycle(go, gp, 1, UPD, psi=psi_d)
        plan, gpos, goffs = refine_positions(plan, go, gp, psi_d, gpos, pos0)
    assert not np.array_equal(start_off, goffs)          # some frames moved to another pixel
    assert np.abs(gpos - pos).max() < 1e-3
    np.testing.assert_array_equal(goffs, oracle.offsets_from_positions(pos, wl.n, wl.obj_shape))
    wrong0 = int((start_off != off_true).any(axis=1).sum())
    wrong = int((goffs != off_true).any(axis=1).sum())
    assert wrong < wrong0


def test_timing_records_only_the_selected_kernel_classes(dev):
    from paper_2008_11511_amd import PtychoError
    from paper_2008_11511_amd._lib import lib
    wl = small("dm256", n=64, k=2, j=20, obj=(160, 160), step=4.0, mask_frac=0.0)
    pb = make_problem(wl, start="ml")
    say("timing class mask")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    psi = plan.psi_init(o, p)
    plan.timing(True, ("rows_inv",))
    plan.dm_cycle(o, p, psi, 3, UPD)
    per = plan.timing_read()
    assert per["rows_inv"][1] == 3 and per["rows_inv"][0] > 0
    assert all(n == 0 for name, (_, n) in per.items() if name != "rows_inv")
    plan.timing(True)
    plan.dm_cycle(o, p, psi, 2, UPD)
    per = plan.timing_read()
    assert per["rows_fwd"][1] == 2 and per["cols"][1] == 2 and per["rows_inv"][1] == 2
    plan.timing(False)
    with pytest.raises(PtychoError):
        from paper_2008_11511_amd._lib import check
        check(lib().ptycho_plan_timing(plan._h, 256))

"""Near-field geometry on the GPU against the FP64 oracle (operator
PropagateNearField in place of FT / IFT in every operator).

Same bar as the far field: relative L2 <= 1e-4 after one cycle or one
gradient, <= 1e-3 after many cycles.  Every case prints its name first.
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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def near(n, k, j, f_pixel=0.02, mask_frac=0.0, seed_offset=0, start="apdm", fxy=None, step=None):
    """A small near-field problem: positions in a square of side `step`
    (default n/2), object n + step + 32, Fresnel number f_pixel per pixel
    (fxy overrides (f_y, f_x))."""
    step = n // 2 if step is None else step
    side = n + step + 32
    f = synth.fresnel_parameter(n, f_pixel)
    wl = small("nf1024", n=n, k=k, j=j, obj=(side, side), step=float(step), mask_frac=mask_frac,
               photons=1e4 * n * n, fresnel=f, seed_offset=seed_offset)
    pb = make_problem(wl, start=start)
    if fxy is not None:
        # the same truth seen at another (anisotropic) distance
        pb.nf = fxy
        pb.iobs = synth.poisson_counts(oracle.simulate_intensity(pb.obj_true, pb.probe_true, pb.offsets, nf=fxy),
                                       wl.seed)
    return pb


def make_plan(pb, dev, stack=0):
    from paper_2008_11511_amd import Plan
    iobs = to_dev(pb.iobs, dev, torch.float32)
    mask = to_dev(pb.mask, dev, torch.uint8) if pb.mask is not None else None
    return Plan(pb.offsets, iobs, mask, pb.wl.n_modes, pb.wl.obj_shape, stack=stack, near_field=pb.nf)


def state(pb, dev):
    return (to_dev(pb.obj0, dev, torch.complex64).contiguous(),
            to_dev(pb.probe0, dev, torch.complex64).contiguous())


@pytest.mark.parametrize("n,k,j,mask", [(8, 1, 9, 0.0), (16, 2, 11, 0.0), (64, 1, 13, 0.05), (128, 3, 7, 0.03),
                                        (256, 1, 5, 0.0), (512, 2, 3, 0.0), (1024, 1, 2, 0.0), (2048, 1, 2, 0.0),
                                        (2048, 2, 1, 0.02)])
def test_near_field_icalc_and_llk_match_oracle(dev, n, k, j, mask):
    pb = near(n, k, j, mask_frac=mask)
    say(f"near field icalc/llk n={n} k={k} j={j}")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    ic_ref = oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets, nf=pb.nf)
    assert rel_l2(ic, ic_ref) < 1e-5
    for model in oracle.LLK_MODELS:
        llk = host(plan.llk(o, p, model=model))
        ref, nobs = oracle.llk(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, model=model, nf=pb.nf)
        assert llk[1] == nobs
        assert abs(llk[0] - ref) <= 1e-4 * abs(ref), model


def test_near_field_anisotropic_distances(dev):
    """Different Fresnel parameters on y and x: catches an axis swap."""
    f = synth.fresnel_parameter(64, 0.02)
    pb = near(64, 2, 9, fxy=(f, 2.5 * f))
    say("near field anisotropic n=64 k=2")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    assert rel_l2(ic, oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets, nf=pb.nf)) < 1e-5
    swapped = oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets, nf=(pb.nf[1], pb.nf[0]))
    assert rel_l2(ic, swapped) > 1e-2
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, UPD, nf=pb.nf)
    assert rel_l2(host(psi), rpsi) < 1e-4
    assert rel_l2(host(o), ro) < 1e-4


@pytest.mark.parametrize("n,k,j,stack", [(16, 2, 13, 5), (64, 1, 17, 0), (128, 3, 9, 4), (256, 1, 6, 0),
                                         (512, 1, 3, 2), (1024, 1, 2, 0), (2048, 1, 3, 2)])
def test_near_field_dm_and_ap_one_cycle(dev, n, k, j, stack):
    pb = near(n, k, j, mask_frac=0.03 if n >= 64 else 0.0)
    say(f"near field DM one cycle n={n} k={k} j={j} stack={stack}")
    plan = make_plan(pb, dev, stack=stack)
    o, p = state(pb, dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, UPD, nf=pb.nf)
    assert rel_l2(host(psi), rpsi) < 1e-4
    assert rel_l2(host(o), ro) < 1e-4
    assert rel_l2(host(p), rp) < 1e-4
    say(f"near field AP one cycle n={n} k={k} j={j} stack={stack}")
    o, p = state(pb, dev)
    psi_ap = torch.empty_like(psi)
    plan.ap_cycle(o, p, 1, UPD, psi=psi_ap)
    ro, rp = oracle.ap_cycle(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, UPD, nf=pb.nf)
    assert rel_l2(host(o), ro) < 1e-4
    assert rel_l2(host(p), rp) < 1e-4


def _oracle_dm(pb, o, p, cycles):
    psi = oracle.psi_init(o, p, pb.offsets)
    for _ in range(cycles):
        o, p, psi = oracle.dm_cycle(o, p, psi, pb.offsets, pb.iobs, pb.mask, UPD, nf=pb.nf)
    return o, p


def test_near_field_dm_many_cycles(dev):
    # 20 positions over a square one frame wide: the oracle's own trajectory
    # moves by about 1e-4 after 50 cycles when its start is perturbed at the
    # fp32 rounding level (checked below to stay 3x under the bar), so the
    # 1e-3 bar measures the kernels, not the conditioning.  (With 12
    # positions over half a frame that spread is 5e-4, the order of the bar.)
    pb = near(64, 1, 20, mask_frac=0.03, step=64)
    say("near field DM 50 cycles n=64 k=1 j=20")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 50, UPD)
    ro, rp = _oracle_dm(pb, pb.obj0, pb.probe0, 50)
    assert rel_l2(host(o), ro) < 1e-3
    assert rel_l2(host(p), rp) < 1e-3
    rng = np.random.default_rng(1)
    po, pp = _oracle_dm(pb, pb.obj0 * (1 + 1e-7 * rng.standard_normal(pb.obj0.shape)),
                        pb.probe0 * (1 + 1e-7 * rng.standard_normal(pb.probe0.shape)), 50)
    assert rel_l2(po, ro) < 3e-4 and rel_l2(pp, rp) < 3e-4


# At 2048 (two frames, the LLK falling 100x in five cycles) the oracle's own
# CG trajectory moves by up to 8e-4 in five cycles from a 1e-7 perturbation
# of its start, so the many-cycle check there covers two cycles.
@pytest.mark.parametrize("n,k,j,cycles", [(64, 1, 11, 5), (256, 2, 5, 5), (2048, 1, 2, 2)])
def test_near_field_ml_grad_linesearch_and_cycles(dev, n, k, j, cycles):
    pb = near(n, k, j, mask_frac=0.03, start="ml")
    say(f"near field ML grad n={n} k={k} j={j}")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    go, gp, llk = plan.ml_grad(o, p)
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert rel_l2(host(go), ro) < 1e-4
    assert rel_l2(host(gp), rp) < 1e-4
    assert abs(host(llk)[0] - rl) < 1e-4 * abs(rl)
    rng = np.random.default_rng(5)
    d_o = (rng.standard_normal(pb.obj0.shape) + 1j * rng.standard_normal(pb.obj0.shape)).astype(np.complex64) * 1e-2
    d_p = (rng.standard_normal(pb.probe0.shape) + 1j * rng.standard_normal(pb.probe0.shape)).astype(np.complex64)
    d_p *= 1e-2 * np.abs(pb.probe0).max()
    say(f"near field ML line search n={n}")
    coef = host(plan.ml_linesearch(o, p, to_dev(d_o, dev, torch.complex64), to_dev(d_p, dev, torch.complex64)))
    r1, r2 = oracle.linesearch_coefs(pb.obj0, pb.probe0, d_o, d_p, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert abs(coef[0] - r1) <= 1e-4 * abs(r1)
    assert abs(coef[1] - r2) <= 1e-4 * abs(r2)
    say(f"near field ML {cycles} cycles n={n}")
    o, p = state(pb, dev)
    st = plan.ml_state()
    hist = torch.zeros(cycles, dtype=torch.float64, device=dev)
    plan.ml_cycle(o, p, st, cycles, UPD, reset=True, hist=hist)
    cg = oracle.CGState()
    ro, rp = pb.obj0, pb.probe0
    for _ in range(cycles):
        ro, rp = oracle.ml_cycle(ro, rp, cg, pb.offsets, pb.iobs, pb.mask, update=UPD, nf=pb.nf)
    # the first entry is one step from the same state (the per-step bar);
    # later ones follow the fp32 trajectory, which the fast LLK descent of
    # the near-field problem amplifies (the many-cycle bar)
    h = host(hist)
    np.testing.assert_allclose(h[0], cg.history[0], rtol=1e-4)
    np.testing.assert_allclose(h, cg.history, rtol=1e-3)
    assert rel_l2(host(o), ro) < 1e-3
    assert rel_l2(host(p), rp) < 1e-3


def test_near_field_zero_distance_sees_the_exit_waves(dev):
    pb = near(32, 1, 5)
    say("near field f=0 n=32")
    from paper_2008_11511_amd import Plan
    plan = Plan(pb.offsets, to_dev(pb.iobs, dev, torch.float32), None, 1, pb.wl.obj_shape, near_field=0.0)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    ref = (np.abs(oracle.exit_waves(pb.obj0, pb.probe0, pb.offsets)) ** 2).sum(axis=1)
    assert rel_l2(ic, ref) < 1e-6


def test_near_field_arguments_are_checked(dev):
    from paper_2008_11511_amd import Plan, PtychoError
    from paper_2008_11511_amd._lib import FLAG_NEAR_FIELD, check, lib
    pb = near(32, 1, 5)
    say("near field argument checks")
    iobs = to_dev(pb.iobs, dev, torch.float32)
    far = Plan(pb.offsets, iobs, None, 1, pb.wl.obj_shape)
    with pytest.raises(PtychoError, match="PTYCHO_FLAG_NEAR_FIELD"):
        far.set_near_field(0.1)
    plan = Plan(pb.offsets, iobs, None, 1, pb.wl.obj_shape, near_field=0.1)
    with pytest.raises(PtychoError, match="non-finite"):
        plan.set_near_field(float("nan"))
    # a near-field plan whose parameters were never set refuses to propagate
    raw = Plan(pb.offsets, iobs, None, 1, pb.wl.obj_shape)
    raw.close()
    import ctypes
    d = plan.desc
    d2 = type(d).from_buffer_copy(d)
    d2.flags = FLAG_NEAR_FIELD
    h = ctypes.c_void_p()
    ws = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device=dev)
    offs = np.ascontiguousarray(pb.offsets, dtype=np.int32)
    check(lib().ptycho_plan(ctypes.byref(d2), offs.ctypes.data, iobs.data_ptr(), None, ws.data_ptr(),
                                   plan.workspace_bytes, torch.cuda.current_stream(dev).cuda_stream,
                                   ctypes.byref(h)))
    try:
        o, p = state(pb, dev)
        out = torch.zeros(2, dtype=torch.float64, device=dev)
        rc = lib().ptycho_llk(h, o.data_ptr(), p.data_ptr(), out.data_ptr())
        assert rc == -1 and b"Fresnel" in lib().ptycho_last_error()
    finally:
        lib().ptycho_plan_destroy(h)


def test_near_field_background_matches_oracle(dev):
    """An incoherent background in natural pixel order, in every operator and
    in the AP refinement, near field."""
    from paper_2008_11511_amd import Plan, UPDATE_BACKGROUND
    side = 64 + 32 + 32
    wl = small("nf1024", n=64, k=2, j=12, obj=(side, side), step=32.0, mask_frac=0.03, photons=1e4 * 64 * 64,
               fresnel=synth.fresnel_parameter(64, 0.02))
    pb = make_problem(wl, start="ml", bg_level=500.0)
    say("near field background n=64 k=2")
    iobs = to_dev(pb.iobs, dev, torch.float32)
    mask = to_dev(pb.mask, dev, torch.uint8)
    plan = Plan(pb.offsets, iobs, mask, 2, wl.obj_shape, near_field=pb.nf, background_update=True)
    bg = to_dev(pb.bg0, dev, torch.float32)
    plan.set_background(bg)
    o, p = state(pb, dev)
    ic = host(plan.icalc(o, p))
    assert rel_l2(ic, oracle.simulate_intensity(pb.obj0, pb.probe0, pb.offsets, bg=pb.bg0, nf=pb.nf)) < 1e-5
    for model in oracle.LLK_MODELS:
        llk = host(plan.llk(o, p, model=model))
        ref, _ = oracle.llk(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, model=model, bg=pb.bg0, nf=pb.nf)
        assert abs(llk[0] - ref) <= 1e-4 * abs(ref), model
    go, gp, _ = plan.ml_grad(o, p)
    ro, rp, _ = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, bg=pb.bg0, nf=pb.nf)
    assert rel_l2(host(go), ro) < 1e-4 and rel_l2(host(gp), rp) < 1e-4
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, bg=pb.bg0, nf=pb.nf)
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4 and rel_l2(host(psi), rpsi) < 1e-4
    say("near field AP background refinement n=64 k=2")
    o, p = state(pb, dev)
    plan.ap_cycle(o, p, 1, UPD | UPDATE_BACKGROUND)
    ro, rp, rb = oracle.ap_cycle(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, UPD | oracle.UPDATE_BACKGROUND,
                                 bg=pb.bg0, nf=pb.nf)
    assert rel_l2(host(bg), rb) < 1e-4
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4


def test_near_field_position_refinement_follows_oracle(dev):
    """AP cycles with position updates in the near field: the rebuilt plans
    keep the geometry, and positions follow the oracle."""
    from paper_2008_11511_amd import Plan
    from paper_2008_11511_amd.plan import refine_positions
    n, side = 64, 64 + 64 + 32
    f = synth.fresnel_parameter(n, 0.02)
    wl = small("nf1024", n=n, k=1, j=20, obj=(side, side), step=64.0, mask_frac=0.0, photons=1e4 * n * n,
               fresnel=f)
    pb = make_problem(wl, start="truth")
    pos_true = synth.random_positions(wl.n_frames, wl.step, wl.seed)
    rng = np.random.default_rng(1)
    err = np.zeros_like(pos_true)
    sel = rng.random(len(pos_true)) < 0.5
    err[sel] = rng.choice([-0.4, 0.4], size=(sel.sum(), 2))
    pos0 = pos_true + err
    say("near field position refinement: 2 AP cycles with position updates")
    pos, o, p = pos0.copy(), pb.obj0, pb.probe0
    for _ in range(2):
        offs = oracle.offsets_from_positions(pos, n, wl.obj_shape)
        psi = oracle.fourier_project(oracle.exit_waves(o, p, offs), pb.iobs, None, nf=f)
        o, p = oracle.overlap_update(o, p, psi, offs, UPD)
        sh, e = oracle.position_shifts(o, p, psi, offs)
        pos = oracle.update_positions(pos, pos0, sh, e)
    gpos = pos0.copy()
    plan = Plan(oracle.offsets_from_positions(gpos, n, wl.obj_shape), to_dev(pb.iobs, dev, torch.float32), None, 1,
                wl.obj_shape, near_field=f)
    go, gp = state(pb, dev)
    psi_d = torch.empty((wl.n_frames, 1, n, n), dtype=torch.complex64, device=dev)
    start_off = plan.offsets.copy()
    for _ in range(2):
        plan.ap_cycle(go, gp, 1, UPD, psi=psi_d)
        plan, gpos, goffs = refine_positions(plan, go, gp, psi_d, gpos, pos0)
        assert plan.near_field == (f, f)
    assert not np.array_equal(start_off, goffs)
    assert np.abs(gpos - pos).max() < 1e-3
    np.testing.assert_array_equal(goffs, oracle.offsets_from_positions(pos, n, wl.obj_shape))


def test_near_field_autograd_matches_oracle_gradient(dev):
    """torch.autograd over the near-field adjoint: loss and gradients against
    the oracle, and a torch optimiser step lowers the likelihood."""
    import paper_2008_11511_amd as P
    pb = near(64, 1, 12, mask_frac=0.03, start="ml")
    say("near field autograd PoissonLLK")
    plan = make_plan(pb, dev)
    o, p = state(pb, dev)
    o.requires_grad_(True)
    p.requires_grad_(True)
    loss = P.poisson_llk(o, p, plan)
    loss.backward()
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert abs(float(loss.detach().cpu()) - rl) < 1e-4 * abs(rl)
    assert rel_l2(host(o.grad), ro) < 1e-4 and rel_l2(host(p.grad), rp) < 1e-4
    # a small gradient step on the object lowers the LLK
    with torch.no_grad():
        o2 = o - 1e-3 * float(np.abs(pb.obj0).max()) / float(o.grad.abs().max()) * o.grad
    assert float(P.poisson_llk(o2, p.detach(), plan).cpu()) < float(loss.detach().cpu())

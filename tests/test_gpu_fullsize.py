"""Parity at the full workload sizes, in the launch configuration bench.py
times (automatic stack size).

* DM, 1000 frames 256x256, 3 modes, 2% mask: one whole cycle against the
  oracle (every output).
* ML, 500 frames 256x256, 3 modes: the full gradient and LLK.
* 4000 frames 512x512, 4 modes, 3% mask, object 4096x4096: the oracle cannot
  run a whole cycle in seconds, so (a) the new exit waves of sampled frames,
  which depend only on their own data, are compared one by one, and (b) the
  truth is a fixed point of an AP cycle on noise-free data (a property that
  holds at any size).
* Near field, 17 frames 2048x2048, one probe: one whole DM cycle and the ML
  gradient against the oracle.
* Sub-pixel positions on the DM scan (1000 frames 256x256, 3 modes): one whole
  DM cycle, then the position shifts from its outputs, and the ML gradient on
  the 500-frame scan, against the oracle's bilinear windows.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from cases import make_problem, rel_l2

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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def test_dm256_full_cycle(dev):
    from paper_2008_11511_amd import Plan
    wl = synth.workload("dm256")
    pb = make_problem(wl, start="ml")
    say("full size DM: 1000 frames 256x256, 3 modes")
    plan = Plan(pb.offsets, torch.from_numpy(pb.iobs).to(dev), torch.from_numpy(pb.mask).to(dev), 3, wl.obj_shape)
    o = torch.from_numpy(pb.obj0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(pb.probe0.astype(np.complex64)).to(dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, 3)
    g_psi = host(psi)
    g_o, g_p = host(o), host(p)
    del psi
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask)
    assert rel_l2(g_psi, rpsi) < 1e-4
    assert rel_l2(g_o, ro) < 1e-4
    assert rel_l2(g_p, rp) < 1e-4


def test_ml256_full_gradient(dev):
    from paper_2008_11511_amd import Plan
    wl = synth.workload("ml256")
    pb = make_problem(wl, start="ml")
    say("full size ML gradient: 500 frames 256x256, 3 modes")
    plan = Plan(pb.offsets, torch.from_numpy(pb.iobs).to(dev), torch.from_numpy(pb.mask).to(dev), 3, wl.obj_shape)
    o = torch.from_numpy(pb.obj0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(pb.probe0.astype(np.complex64)).to(dev)
    g_o, g_p, llk = plan.ml_grad(o, p)
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask)
    assert rel_l2(host(g_o), ro) < 1e-4
    assert rel_l2(host(g_p), rp) < 1e-4
    assert abs(host(llk)[0] - rl) < 1e-4 * abs(rl)


def test_apdm512_sampled_frames_and_fixed_point(dev):
    from paper_2008_11511_amd import Plan
    wl = synth.workload("apdm512")
    say("full size 4000 frames 512x512, 4 modes: host inputs")
    obj = synth.object_truth(wl.obj_shape, wl.seed)
    probe = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
    offs = oracle.offsets_from_positions(synth.spiral_positions(wl.n_frames, wl.step), wl.n, wl.obj_shape)
    probe = probe * synth.probe_photon_scale(obj, probe, offs, wl.photons)
    mask = synth.gap_mask(wl.n, wl.mask_frac, wl.seed)
    o_t = torch.from_numpy(obj.astype(np.complex64)).to(dev)
    p_t = torch.from_numpy(probe.astype(np.complex64)).to(dev)
    mask_d = torch.from_numpy(mask).to(dev)

    # (b) fixed point: noise-free data from the forward model, start at the truth
    say("apdm512: forward model and AP fixed point")
    zero = torch.zeros((wl.n_frames, wl.n, wl.n), dtype=torch.float32, device=dev)
    inten = Plan(offs, zero, None, wl.n_modes, wl.obj_shape).icalc(o_t, p_t)
    del zero
    plan = Plan(offs, inten, mask_d, wl.n_modes, wl.obj_shape)
    o1, p1 = o_t.clone(), p_t.clone()
    psi = torch.empty((wl.n_frames, wl.n_modes, wl.n, wl.n), dtype=torch.complex64, device=dev)
    plan.ap_cycle(o1, p1, 1, 3, psi=psi)
    assert rel_l2(host(o1), obj.astype(np.complex64)) < 1e-4
    assert rel_l2(host(p1), probe.astype(np.complex64)) < 1e-4
    del plan

    # (a) sampled frames: Poisson data, the sampled frames' data from the oracle
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(wl.n_frames, 6, replace=False))
    gen = torch.Generator(device=dev)
    gen.manual_seed(wl.seed)
    iobs = torch.poisson(inten, generator=gen)
    del inten
    o0 = synth.perturb_object(obj, wl.seed).astype(np.complex64).astype(np.complex128)
    p0 = synth.perturb_probe(probe, wl.seed).astype(np.complex64).astype(np.complex128)
    ref_i = synth.poisson_counts(oracle.simulate_intensity(obj, probe, offs[sample]), wl.seed + 99)
    iobs[torch.from_numpy(sample).to(dev)] = torch.from_numpy(ref_i).to(dev)
    say("apdm512: one DM cycle on the GPU")
    plan = Plan(offs, iobs.contiguous(), mask_d, wl.n_modes, wl.obj_shape)
    o = torch.from_numpy(o0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(p0.astype(np.complex64)).to(dev)
    plan.psi_init(o, p, psi)
    plan.dm_cycle(o, p, psi, 1, 3)
    got = host(psi[torch.from_numpy(sample).to(dev)])
    psi0 = oracle.psi_init(o0, p0, offs[sample])
    _, _, ref = oracle.dm_cycle(o0, p0, psi0, offs[sample], ref_i, mask, update=0)
    for i in range(len(sample)):
        assert rel_l2(got[i], ref[i]) < 1e-4, sample[i]


def test_nf2048_full_dm_cycle_and_gradient(dev):
    """Near field, 17 frames 2048x2048, one probe, object 2368x2368: one whole
    DM cycle and the ML gradient against the oracle (every output)."""
    from paper_2008_11511_amd import Plan
    wl = synth.workload("nf2048")
    pb = make_problem(wl, start="ml")
    say("full size near field: 17 frames 2048x2048, 1 mode")
    plan = Plan(pb.offsets, torch.from_numpy(pb.iobs).to(dev), None, 1, wl.obj_shape, near_field=wl.fresnel)
    o = torch.from_numpy(pb.obj0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(pb.probe0.astype(np.complex64)).to(dev)
    g_o, g_p, llk = plan.ml_grad(o, p)
    gg_o, gg_p, gl = host(g_o), host(g_p), host(llk)[0]
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, 3)
    g_psi, d_o, d_p = host(psi), host(o), host(p)
    del psi, plan
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert rel_l2(gg_o, ro) < 1e-4
    assert rel_l2(gg_p, rp) < 1e-4
    assert abs(gl - rl) < 1e-4 * abs(rl)
    del ro, rp
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert rel_l2(g_psi, rpsi) < 1e-4
    assert rel_l2(d_o, ro) < 1e-4
    assert rel_l2(d_p, rp) < 1e-4


def _subpixel_positions(pb, wl, seed):
    """Real positions whose corners are the scan's integer corners plus a
    fraction in [0, 1) on each axis (windows well inside the object), and
    Poisson data simulated at those positions.  Data taken at the integer
    corners would leave the model far from the data at the sub-pixel ones,
    where the probe gradient is ill-conditioned: a 1e-7 relative change of
    the object and probe then moves the oracle's own probe gradient by 3e-4,
    against 1e-6 with consistent data."""
    rng = np.random.default_rng(seed)
    t = pb.offsets.astype(np.float64) + rng.uniform(0.0, 1.0, (wl.n_frames, 2))
    pos = t - np.array(wl.obj_shape) / 2.0 + wl.n / 2.0
    offs, frac = oracle.windows_from_positions(pos, wl.n, wl.obj_shape)
    np.testing.assert_array_equal(offs, pb.offsets)
    inten = oracle.simulate_intensity(pb.obj_true, pb.probe_true, offs, frac=frac)
    iobs = synth.poisson_counts(inten, wl.seed).astype(np.float32)
    return pos, frac, iobs


def test_dm256_subpixel_full_cycle_and_shifts(dev):
    from paper_2008_11511_amd import Plan
    wl = synth.workload("dm256")
    pb = make_problem(wl, start="ml")
    pos, frac, iobs = _subpixel_positions(pb, wl, 11)
    say("full size DM with sub-pixel windows: 1000 frames 256x256, 3 modes")
    plan = Plan.with_positions(pos, torch.from_numpy(iobs).to(dev), torch.from_numpy(pb.mask).to(dev), 3,
                               wl.obj_shape, max_shift=1.0)
    o = torch.from_numpy(pb.obj0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(pb.probe0.astype(np.complex64)).to(dev)
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, 3)
    g_psi, g_o, g_p = host(psi), host(o), host(p)
    psi0 = oracle.psi_init(pb.obj0, pb.probe0, pb.offsets, frac)
    ro, rp, rpsi = oracle.dm_cycle(pb.obj0, pb.probe0, psi0, pb.offsets, iobs, pb.mask, frac=frac)
    assert rel_l2(g_psi, rpsi) < 1e-4
    assert rel_l2(g_o, ro) < 1e-4
    assert rel_l2(g_p, rp) < 1e-4
    say("position shifts from the cycle's outputs, same inputs on both sides")
    got = host(plan.position_shifts(o, p, psi))
    del psi
    ref, e_ref = oracle.position_shifts(g_o.astype(np.complex64).astype(np.complex128),
                                        g_p.astype(np.complex64).astype(np.complex128),
                                        g_psi.astype(np.complex64).astype(np.complex128), pb.offsets, frac)
    scale = np.abs(ref).max()
    assert scale > 0
    assert np.abs(got[:, :2] - ref).max() <= 1e-3 * scale
    np.testing.assert_allclose(got[:, 2], e_ref, rtol=1e-4)


def test_ml256_subpixel_full_gradient(dev):
    from paper_2008_11511_amd import Plan
    wl = synth.workload("ml256")
    pb = make_problem(wl, start="ml")
    pos, frac, iobs = _subpixel_positions(pb, wl, 12)
    say("full size ML gradient with sub-pixel windows: 500 frames 256x256, 3 modes")
    plan = Plan.with_positions(pos, torch.from_numpy(iobs).to(dev), torch.from_numpy(pb.mask).to(dev), 3,
                               wl.obj_shape, max_shift=1.0)
    o = torch.from_numpy(pb.obj0.astype(np.complex64)).to(dev)
    p = torch.from_numpy(pb.probe0.astype(np.complex64)).to(dev)
    g_o, g_p, llk = plan.ml_grad(o, p)
    ro, rp, rl = oracle.ml_grad(pb.obj0, pb.probe0, pb.offsets, iobs, pb.mask, frac=frac)
    assert rel_l2(host(g_o), ro) < 1e-4
    assert rel_l2(host(g_p), rp) < 1e-4
    assert abs(host(llk)[0] - rl) < 1e-4 * abs(rl)

"""Degenerate inputs on the GPU against the FP64 oracle: a single frame that
covers the whole object, frames at the four corners of a non-square object,
an all-bad mask, and frames with no photons; far and near field."""
import sys

import numpy as np
import pytest

import oracle
import synth
from cases import rel_l2

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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy().astype(np.complex128 if t.is_complex() else np.float64)


def td(a, dev, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev, dtype)


def problem(n, k, offs, obj_shape, nf=None, seed=3, photons=1e6):
    """Truth, Poisson data from the oracle, and a start near the truth."""
    obj = synth.object_truth(obj_shape, seed)
    probe = synth.probe_modes(n, k, seed) if nf is None else synth.near_field_probe(n, k, seed)
    offs = np.asarray(offs, dtype=np.int32)
    probe = probe * synth.probe_photon_scale(obj, probe, offs, photons)
    iobs = synth.poisson_counts(oracle.simulate_intensity(obj, probe, offs, nf=nf), seed)
    o0 = synth.perturb_object(obj, seed).astype(np.complex64).astype(np.complex128)
    p0 = synth.perturb_probe(probe, seed).astype(np.complex64).astype(np.complex128)
    return offs, iobs, o0, p0


def check_all(dev, n, k, offs, obj_shape, iobs, mask, o0, p0, nf=None):
    """DM and AP cycles, LLK and the ML gradient against the oracle."""
    from paper_2008_11511_amd import Plan
    plan = Plan(offs, td(iobs, dev, torch.float32), td(mask, dev, torch.uint8) if mask is not None else None, k,
                obj_shape, near_field=nf)
    o, p = td(o0, dev, torch.complex64), td(p0, dev, torch.complex64)
    llk = host(plan.llk(o, p))
    rl, nobs = oracle.llk(o0, p0, offs, iobs, mask, nf=nf)
    assert llk[1] == nobs
    assert abs(llk[0] - rl) <= 1e-4 * max(abs(rl), 1e-30) + 1e-6
    go, gp, _ = plan.ml_grad(o, p)
    ro, rp, _ = oracle.ml_grad(o0, p0, offs, iobs, mask, nf=nf)
    scale = max(np.linalg.norm(ro), np.linalg.norm(rp), 1e-30)
    assert np.linalg.norm(host(go) - ro) <= 1e-4 * scale
    assert np.linalg.norm(host(gp) - rp) <= 1e-4 * scale
    psi = plan.psi_init(o, p)
    plan.dm_cycle(o, p, psi, 1, UPD)
    psi0 = oracle.psi_init(o0, p0, offs)
    ro, rp, rpsi = oracle.dm_cycle(o0, p0, psi0, offs, iobs, mask, UPD, nf=nf)
    # relative to the exit waves' scale: with no photons the new exit waves
    # are exactly zero in the oracle and fp32 rounding of Phi - Phi on the GPU
    assert np.linalg.norm(host(psi) - rpsi) <= 1e-4 * max(np.linalg.norm(rpsi), np.linalg.norm(psi0))
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4
    o, p = td(o0, dev, torch.complex64), td(p0, dev, torch.complex64)
    plan.ap_cycle(o, p, 1, UPD, psi=psi)
    ro, rp = oracle.ap_cycle(o0, p0, offs, iobs, mask, UPD, nf=nf)
    assert rel_l2(host(o), ro) < 1e-4 and rel_l2(host(p), rp) < 1e-4
    return plan


@pytest.mark.parametrize("geometry", ["far", "near"])
def test_one_frame_covering_the_whole_object(dev, geometry):
    n, k = 64, 2
    nf = synth.fresnel_parameter(n, 0.02) if geometry == "near" else None
    say(f"edge: one frame = whole object ({geometry})")
    offs, iobs, o0, p0 = problem(n, k, [[0, 0]], (n, n), nf)
    check_all(dev, n, k, offs, (n, n), iobs, None, o0, p0, nf)


@pytest.mark.parametrize("geometry", ["far", "near"])
def test_frames_at_the_corners_of_a_non_square_object(dev, geometry):
    n, k = 32, 1
    ny, nx = n + 45, n + 13
    nf = synth.fresnel_parameter(n, 0.02) if geometry == "near" else None
    say(f"edge: corner frames, object {ny}x{nx} ({geometry})")
    offs, iobs, o0, p0 = problem(n, k, [[0, 0], [0, nx - n], [ny - n, 0], [ny - n, nx - n], [20, 7]], (ny, nx), nf)
    check_all(dev, n, k, offs, (ny, nx), iobs, synth.gap_mask(n, 0.2, 5, fft_order=nf is None), o0, p0, nf)


def test_all_bad_mask_leaves_the_views_and_counts_nothing(dev):
    from paper_2008_11511_amd import Plan
    n, k = 32, 2
    say("edge: every pixel masked")
    offs, iobs, o0, p0 = problem(n, k, [[0, 0], [3, 5], [9, 2]], (48, 48))
    mask = np.ones((n, n), dtype=np.uint8)
    plan = Plan(offs, td(iobs, dev, torch.float32), td(mask, dev, torch.uint8), k, (48, 48))
    o, p = td(o0, dev, torch.complex64), td(p0, dev, torch.complex64)
    llk = host(plan.llk(o, p))
    assert llk[0] == 0.0 and llk[1] == 0.0
    go, gp, _ = plan.ml_grad(o, p)
    assert not host(go).any() and not host(gp).any()
    # no Fourier constraint: the DM update returns the views of the same state
    psi = td(oracle.psi_init(o0, p0, offs) * 1.5, dev, torch.complex64)
    plan.dm_cycle(o, p, psi, 1, 0)
    np.testing.assert_allclose(host(psi), oracle.exit_waves(o0.astype(np.complex64), p0.astype(np.complex64), offs),
                               atol=1e-5 * np.abs(p0).max())


def test_frames_without_photons(dev):
    n, k = 32, 1
    say("edge: zero photons in every frame")
    offs, _, o0, p0 = problem(n, k, [[0, 0], [4, 6], [8, 1]], (48, 48))
    iobs = np.zeros((3, n, n), dtype=np.float32)
    plan = check_all(dev, n, k, offs, (48, 48), iobs, None, o0, p0)
    # the LLK is the total calculated intensity, the projection empties the frames
    o, p = td(o0, dev, torch.complex64), td(p0, dev, torch.complex64)
    ic = host(plan.icalc(o, p))
    np.testing.assert_allclose(host(plan.llk(o, p))[0], ic.sum(), rtol=1e-5)
    psi = plan.psi_init(o, p)
    plan.ap_cycle(o, p, 1, 0, psi=psi)
    assert np.abs(host(psi)).max() <= 1e-6 * np.abs(p0).max()

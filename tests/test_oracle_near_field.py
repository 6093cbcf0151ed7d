"""Pins of the oracle's near-field geometry (operator PropagateNearField and
the near-field form of PropagateApplyAmplitude), independent of the oracle's
own formulas:

* the paraxial Gaussian beam, whose propagation has a closed form
  (q-parameter 1 + i z/z_R per axis), with different Fresnel parameters on
  the two axes (catches a sign, an axis swap or a wrong frequency index);
* the Talbot self-image of a periodic field, and the half-period shift at
  half the Talbot distance;
* unitarity, inverse and composition;
* the fixed point at the truth, zero likelihood there, and finite
  differences of the gradient and of the line search, with near-field data.
"""
import math

import numpy as np
import pytest

import oracle


def crandn(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _gauss_1d(n, w0, a):
    """Paraxial Gaussian beam along one axis after propagating z = a z_R:
    (1 + i a)^(-1/2) exp(-y^2 / (w0^2 (1 + i a)))."""
    y = np.arange(n) - n // 2
    q = 1.0 + 1j * a
    return np.exp(-(y ** 2) / (w0 ** 2 * q)) / np.sqrt(q)


@pytest.mark.parametrize("ay, ax", [(0.5, 0.5), (0.8, 0.25), (-0.4, 0.6)])
def test_gaussian_beam_closed_form(ay, ax):
    n, w0 = 128, 6.0
    # with unit pixels, z / z_R = lambda z / (pi w0^2) and f = pi lambda z / N^2
    fy, fx = ay * math.pi ** 2 * w0 ** 2 / n ** 2, ax * math.pi ** 2 * w0 ** 2 / n ** 2
    u0 = np.outer(_gauss_1d(n, w0, 0.0), _gauss_1d(n, w0, 0.0))
    want = np.outer(_gauss_1d(n, w0, ay), _gauss_1d(n, w0, ax))
    got = oracle.propagate_near_field(u0, (fy, fx))
    assert np.abs(got - want).max() < 1e-10
    # back-propagation returns the waist
    assert np.abs(oracle.propagate_near_field(want, (fy, fx), -1) - u0).max() < 1e-10


def test_gaussian_beam_spreads_with_the_right_width():
    n, w0, a = 256, 5.0, 2.0
    f = a * math.pi ** 2 * w0 ** 2 / n ** 2
    u0 = np.outer(_gauss_1d(n, w0, 0.0), _gauss_1d(n, w0, 0.0))
    i1 = np.abs(oracle.propagate_near_field(u0, f)) ** 2
    y = np.arange(n) - n // 2
    prof = i1.sum(axis=1) / i1.sum()
    # intensity profile exp(-2 y^2 / w^2), w = w0 sqrt(1 + a^2): second moment w^2 / 4
    np.testing.assert_allclose((prof * y ** 2).sum(), w0 ** 2 * (1 + a * a) / 4.0, rtol=1e-9)


@pytest.mark.parametrize("p", [4, 8, 16])
def test_talbot_self_image_and_half_period_shift(p):
    n = 64
    rng = np.random.default_rng(p)
    cell = crandn(rng, p, p)
    u0 = np.tile(cell, (n // p, n // p))
    f_talbot = 2.0 * math.pi * p * p / (n * n)
    np.testing.assert_allclose(oracle.propagate_near_field(u0, f_talbot), u0, atol=1e-11)
    half = oracle.propagate_near_field(u0, f_talbot / 2.0)
    np.testing.assert_allclose(half, np.roll(u0, (p // 2, p // 2), axis=(0, 1)), atol=1e-11)
    # different periods on the two axes: Talbot along y only
    u1 = np.tile(crandn(rng, p, n), (n // p, 1))
    np.testing.assert_allclose(oracle.propagate_near_field(u1, (f_talbot, 0.0)), u1, atol=1e-11)


def test_propagation_is_unitary_invertible_and_composes():
    rng = np.random.default_rng(5)
    x = crandn(rng, 3, 32, 32)
    f1, f2 = (0.013, 0.021), (-0.004, 0.05)
    y = oracle.propagate_near_field(x, f1)
    np.testing.assert_allclose(np.linalg.norm(y), np.linalg.norm(x), rtol=1e-13)
    np.testing.assert_allclose(oracle.propagate_near_field(y, f1, -1), x, atol=1e-12)
    both = oracle.propagate_near_field(oracle.propagate_near_field(x, f1), f2)
    np.testing.assert_allclose(both, oracle.propagate_near_field(x, (f1[0] + f2[0], f1[1] + f2[1])), atol=1e-12)
    np.testing.assert_allclose(oracle.propagate_near_field(x, 0.0), x, atol=1e-13)
    # adjoint: <D x, z> = <x, D^-1 z>
    z = crandn(rng, 3, 32, 32)
    np.testing.assert_allclose(np.vdot(y, z), np.vdot(x, oracle.propagate_near_field(z, f1, -1)), rtol=1e-12)


def near_problem(n=16, k=2, j=5, obj=(28, 28), seed=7, f=(0.02, 0.03), mask=True, noiseless=True):
    rng = np.random.default_rng(seed)
    o = (0.8 + 0.2 * rng.random(obj)) * np.exp(1j * rng.uniform(-1, 1, obj))
    p = crandn(rng, k, n, n) * 3.0
    offs = np.stack([rng.integers(0, obj[0] - n + 1, j), rng.integers(0, obj[1] - n + 1, j)],
                    axis=1).astype(np.int32)
    inten = oracle.simulate_intensity(o, p, offs, nf=f)
    iobs = inten if noiseless else rng.poisson(inten).astype(np.float64)
    m = None
    if mask:
        m = np.zeros((n, n), dtype=np.uint8)
        m[:, 3] = 1
        m[9, :] = 1
    return o, p, offs, iobs, m, f


def test_near_field_data_differ_from_far_field_and_zero_distance_is_real_space():
    o, p, offs, _, _, f = near_problem()
    near = oracle.simulate_intensity(o, p, offs, nf=f)
    far = oracle.simulate_intensity(o, p, offs)
    assert np.abs(near - far).max() > 0.1 * far.max()
    # at zero distance the detector sees the exit waves themselves
    at0 = oracle.simulate_intensity(o, p, offs, nf=0.0)
    np.testing.assert_allclose(at0, (np.abs(oracle.exit_waves(o, p, offs)) ** 2).sum(axis=1), rtol=1e-12)


def test_near_field_truth_is_a_fixed_point_and_llk_vanishes():
    o, p, offs, iobs, m, f = near_problem()
    o1, p1 = oracle.ap_cycle(o, p, offs, iobs, m, nf=f)
    assert np.abs(o1 - o).max() < 1e-12 * np.abs(o).max()
    assert np.abs(p1 - p).max() < 1e-12 * np.abs(p).max()
    psi = oracle.psi_init(o, p, offs)
    o2, p2, psi2 = oracle.dm_cycle(o, p, psi, offs, iobs, m, nf=f)
    assert np.abs(psi2 - psi).max() < 1e-12 * np.abs(psi).max()
    assert np.abs(o2 - o).max() < 1e-12 * np.abs(o).max()
    assert abs(oracle.llk(o, p, offs, iobs, m, nf=f)[0]) < 1e-9 * iobs.sum()
    # the far-field model does not fit near-field data
    assert oracle.llk(o, p, offs, iobs, m)[0] > 1e-2 * iobs.sum()
    g_o, g_p, _ = oracle.ml_grad(o, p, offs, iobs, m, nf=f)
    g2_o, _, _ = oracle.ml_grad(o * 1.01, p, offs, iobs, m, nf=f)
    assert np.linalg.norm(g_o) < 1e-10 * np.linalg.norm(g2_o)


def test_near_field_projection_matches_amplitudes_in_the_detector_plane():
    o, p, offs, iobs, m, f = near_problem(noiseless=False, seed=9)
    x = oracle.exit_waves(o * np.exp(0.3j), p * 1.2, offs)
    y = oracle.fourier_project(x, iobs, None, nf=f)
    det = oracle.propagate_near_field(y, f)
    np.testing.assert_allclose((np.abs(det) ** 2).sum(axis=1), iobs, rtol=1e-9, atol=1e-9)
    # projecting twice changes nothing
    np.testing.assert_allclose(oracle.fourier_project(y, iobs, None, nf=f), y, atol=1e-9)


def _fd(fun, x, g, idx, h):
    for i in idx:
        e = np.zeros_like(x)
        e.flat[i] = h
        re = (fun(x + e) - fun(x - e)) / (2 * h)
        im = (fun(x + 1j * e) - fun(x - 1j * e)) / (2 * h)
        np.testing.assert_allclose(g.flat[i].real, re, rtol=2e-5, atol=1e-6 * abs(g).max())
        np.testing.assert_allclose(g.flat[i].imag, im, rtol=2e-5, atol=1e-6 * abs(g).max())


def test_near_field_gradient_and_line_search_match_central_differences():
    o, p, offs, iobs, m, f = near_problem(noiseless=False, seed=11)
    o0 = o * np.exp(0.2j * np.cos(np.arange(o.size).reshape(o.shape)))
    p0 = p * 1.05
    g_o, g_p, lsum = oracle.ml_grad(o0, p0, offs, iobs, m, nf=f)
    np.testing.assert_allclose(lsum, oracle.llk(o0, p0, offs, iobs, m, nf=f)[0], rtol=1e-12)
    rng = np.random.default_rng(3)
    lo = lambda x: oracle.llk(x, p0, offs, iobs, m, nf=f)[0]
    lp = lambda x: oracle.llk(o0, x, offs, iobs, m, nf=f)[0]
    illum = np.flatnonzero(abs(g_o) > 0)
    _fd(lo, o0, g_o, rng.choice(illum, 8, replace=False), 1e-3 * np.sqrt((abs(o0) ** 2).mean()))
    _fd(lp, p0, g_p, rng.choice(p0.size, 8, replace=False), 1e-3 * np.sqrt((abs(p0) ** 2).mean()))
    d_o = crandn(rng, *o.shape) * 1e-2
    d_p = crandn(rng, *p.shape) * 1e-2
    l1, l2 = oracle.linesearch_coefs(o0, p0, d_o, d_p, offs, iobs, m, nf=f)
    fl = lambda gm: oracle.llk(o0 + gm * d_o, p0 + gm * d_p, offs, iobs, m, nf=f)[0]
    h = 1e-3
    np.testing.assert_allclose(l1, (fl(h) - fl(-h)) / (2 * h), rtol=1e-6)
    np.testing.assert_allclose(l2, (fl(h) - 2 * fl(0) + fl(-h)) / h ** 2, rtol=1e-4)


def test_near_field_generators():
    import synth
    for name in ("nf2048", "nf1024"):
        wl = synth.workload(name)
        assert wl.geometry == "near" and wl.n_modes == 1 and wl.n_frames == 17
        np.testing.assert_allclose(wl.fresnel * wl.n ** 2 * synth.NEAR_FIELD_NF_PIXEL, math.pi, rtol=1e-12)
        pos = synth.random_positions(wl.n_frames, wl.step, wl.seed)
        offs = oracle.offsets_from_positions(pos, wl.n, wl.obj_shape)
        assert offs.min() >= 0 and offs.max() <= wl.obj_shape[0] - wl.n
    p = synth.near_field_probe(64, 3, 5)
    np.testing.assert_allclose((np.abs(p) ** 2).sum(axis=(1, 2)), synth.mode_weights(3), rtol=1e-12)
    g = np.einsum("kyx,lyx->kl", p.conj(), p)
    np.testing.assert_allclose(g - np.diag(np.diag(g)), 0.0, atol=1e-12)
    # broad illumination: most of the frame is lit
    i0 = np.abs(p[0]) ** 2
    assert (i0 > 0.1 * i0.mean()).mean() > 0.7
    m = synth.gap_mask(64, 0.1, 3, fft_order=False)
    np.testing.assert_array_equal(np.fft.ifftshift(m), synth.gap_mask(64, 0.1, 3))


def test_near_field_dm_reduces_the_likelihood():
    """Sanity (not parity): DM from the usual start fits near-field data."""
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    import synth
    from cases import make_problem, small
    wl = small("nf1024", n=32, j=6, obj=(72, 72), step=24.0, photons=1e4 * 32 * 32,
               fresnel=synth.fresnel_parameter(32, 0.02))
    pb = make_problem(wl)
    o, p = pb.obj0, pb.probe0
    psi = oracle.psi_init(o, p, pb.offsets)
    l0 = oracle.llk(o, p, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)[0]
    for _ in range(15):
        o, p, psi = oracle.dm_cycle(o, p, psi, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)
    assert oracle.llk(o, p, pb.offsets, pb.iobs, pb.mask, nf=pb.nf)[0] < 0.2 * l0


@pytest.mark.parametrize("n", [4, 6, 8])
def test_propagation_is_a_circular_convolution_with_the_fresnel_kernel(n):
    """Brute force on tiny frames: D x equals the circular convolution of x
    with h = inverse DFT of Q, every sum written out (no FFT)."""
    fy, fx = 0.37, -0.21
    rng = np.random.default_rng(n)
    x = crandn(rng, n, n)
    us = [u if u < n / 2 else u - n for u in range(n)]
    q = [[np.exp(-1j * (fy * us[u] ** 2 + fx * us[v] ** 2)) for v in range(n)] for u in range(n)]
    h = np.zeros((n, n), dtype=np.complex128)
    for y in range(n):
        for xx in range(n):
            h[y, xx] = sum(q[u][v] * np.exp(2j * np.pi * (u * y + v * xx) / n)
                           for u in range(n) for v in range(n)) / (n * n)
    want = np.zeros((n, n), dtype=np.complex128)
    for y in range(n):
        for xx in range(n):
            want[y, xx] = sum(h[(y - a) % n, (xx - b) % n] * x[a, b] for a in range(n) for b in range(n))
    np.testing.assert_allclose(oracle.propagate_near_field(x, (fy, fx)), want, atol=1e-12)


def test_golden_scalar_dm_cases_hold_in_the_near_field():
    """With 1x1 frames the only frequency is 0, where the transfer function
    is 1: the hand-worked DM cases of the far field hold unchanged."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "scalar_cases.json")) as f:
        cases = json.load(f)
    for c in cases["dm"]:
        o = np.array([[complex(*c["obj"])]])
        p = np.array([[[complex(*c["probe"])]]])
        psi = np.array([[[[complex(*c["psi"])]]]])
        offs = np.zeros((1, 2), np.int32)
        _, _, psi1 = oracle.dm_cycle(o, p, psi, offs, np.array([[[c["iobs"]]]]), None, nf=(0.7, -1.3))
        assert abs(psi1[0, 0, 0, 0] - complex(*c["psi_new"])) < 1e-12, c

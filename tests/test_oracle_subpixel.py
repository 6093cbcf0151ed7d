"""Pins of the oracle's sub-pixel windows (refined positions are real numbers;
a window at a fractional corner views the object by bilinear interpolation).

* integer corners (zero fractions) reproduce the integer-window operators
  exactly;
* a 2D plane wave viewed at a fractional corner is the exactly shifted plane
  wave times the transfer function of linear interpolation,
  (1 - f + f e^{ik}) e^{-ikf} per axis (the Fourier shift theorem for the
  interpolated view), and an object linear in y and x is viewed exactly;
* views_adjoint is the adjoint of views (<S x, y> = <x, S^T y>) and the object
  denominator equals the row sums of the dense normal matrix
  sum_j S_j^T diag(sum_k |P_k|^2) S_j, built by brute force;
* the ML gradient and the line-search coefficients with sub-pixel windows
  against central differences of the likelihood;
* position shifts recover a known sub-pixel displacement, from AP exit waves
  and from the ML gradient's back-propagated wave.
"""
import numpy as np
import pytest

import oracle
from test_oracle_pins import crandn


def test_windows_from_positions_split_the_corner():
    offs, frac = oracle.windows_from_positions(np.array([[0.0, 0.0], [1.25, -2.5], [-0.1, 3.0]]), 8, (20, 24))
    # corner = centre + p - N/2: (10 - 4, 12 - 4) = (6, 8)
    np.testing.assert_array_equal(offs, [[6, 8], [7, 5], [5, 11]])
    np.testing.assert_allclose(frac, [[0.0, 0.0], [0.25, 0.5], [0.9, 0.0]], atol=1e-12)
    with pytest.raises(ValueError):
        oracle.windows_from_positions(np.array([[-6.5, 0.0]]), 8, (20, 24))
    with pytest.raises(ValueError):
        oracle.windows_from_positions(np.array([[0.0, 8.01]]), 8, (20, 24))
    # the last corner of the object is allowed (its fraction is then zero)
    offs, frac = oracle.windows_from_positions(np.array([[6.0, 8.0]]), 8, (20, 24))
    np.testing.assert_array_equal(offs, [[12, 16]])
    assert not frac.any()


def _problem(seed=3, j=6, n=8, obj=(24, 24), k=2):
    rng = np.random.default_rng(seed)
    o = (0.8 + 0.2 * rng.random(obj)) * np.exp(1j * rng.uniform(-1, 1, obj))
    p = crandn(k, n, n, rng=rng) * 2.0
    t = np.stack([rng.uniform(0, obj[0] - n, j), rng.uniform(0, obj[1] - n, j)], axis=1)
    offs = np.floor(t).astype(np.int32)
    return o, p, offs, t - offs


def test_zero_fractions_reproduce_the_integer_windows_exactly():
    o, p, offs, _ = _problem()
    zero = np.zeros((len(offs), 2))
    np.testing.assert_array_equal(oracle.views(o, offs, 8, zero), oracle.views(o, offs, 8))
    psi = crandn(len(offs), 2, 8, 8)
    for a, b in zip(oracle.overlap_sums(psi, o, p, offs, zero), oracle.overlap_sums(psi, o, p, offs)):
        np.testing.assert_array_equal(a, b)
    iobs = oracle.simulate_intensity(o * 1.1, p, offs)
    for a, b in zip(oracle.ml_grad(o, p, offs, iobs, None, frac=zero), oracle.ml_grad(o, p, offs, iobs, None)):
        np.testing.assert_array_equal(a, b)


def test_bilinear_view_of_a_plane_wave_is_the_shifted_wave_times_the_interpolation_transfer():
    ny, nx, n = 32, 32, 8
    ky, kx = 0.7, -1.3
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    o = np.exp(1j * (ky * yy + kx * xx))
    offs = np.array([[5, 9], [11, 3]], np.int32)
    frac = np.array([[0.3, 0.8], [0.55, 0.05]])
    v = oracle.views(o, offs, n, frac)
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for j in range(2):
        ty, tx = offs[j] + frac[j]
        exact = np.exp(1j * (ky * (ty + y) + kx * (tx + x)))
        h = lambda f, k: (1 - f + f * np.exp(1j * k)) * np.exp(-1j * k * f)
        np.testing.assert_allclose(v[j], exact * h(frac[j, 0], ky) * h(frac[j, 1], kx), rtol=0, atol=1e-13)


def test_bilinear_view_of_a_linear_object_is_exact():
    yy, xx = np.meshgrid(np.arange(20.0), np.arange(20.0), indexing="ij")
    o = (0.3 + 0.1j) + (0.02 - 0.05j) * yy + (0.07 + 0.01j) * xx
    offs = np.array([[3, 4]], np.int32)
    frac = np.array([[0.37, 0.91]])
    y, x = np.meshgrid(np.arange(8.0), np.arange(8.0), indexing="ij")
    ty, tx = 3.37 + y, 4.91 + x
    np.testing.assert_allclose(oracle.views(o, offs, 8, frac)[0],
                               (0.3 + 0.1j) + (0.02 - 0.05j) * ty + (0.07 + 0.01j) * tx, atol=1e-13)


def test_views_adjoint_is_the_adjoint_and_the_denominator_the_normal_row_sums():
    o, p, offs, frac = _problem(j=4, obj=(16, 16))
    n, shape = 8, o.shape
    x = crandn(*shape)
    y = crandn(len(offs), n, n)
    lhs = np.vdot(oracle.views(x, offs, n, frac), y)
    rhs = np.vdot(x, oracle.views_adjoint(y, offs, shape, frac))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # dense S_j: column i = the views of the i-th unit object
    m = shape[0] * shape[1]
    s = np.zeros((len(offs), n * n, m))
    for i in range(m):
        e = np.zeros(m)
        e[i] = 1.0
        s[:, :, i] = oracle.views(e.reshape(shape), offs, n, frac).reshape(len(offs), n * n).real
    d = (np.abs(p) ** 2).sum(axis=0).ravel()
    normal = sum(s[j].T @ (d[:, None] * s[j]) for j in range(len(offs)))
    _, den_o, _, _ = oracle.overlap_sums(crandn(len(offs), 2, n, n), o, p, offs, frac)
    np.testing.assert_allclose(den_o.ravel(), normal.sum(axis=1), rtol=1e-12, atol=1e-12)
    # for integer windows the normal matrix is diagonal and equals den_o exactly
    zero = np.zeros_like(frac)
    s0 = np.stack([np.stack([oracle.views(np.eye(m)[i].reshape(shape), offs, n, zero)[j].ravel().real
                             for i in range(m)], axis=1) for j in range(len(offs))])
    n0 = sum(s0[j].T @ (d[:, None] * s0[j]) for j in range(len(offs)))
    assert np.count_nonzero(n0 - np.diag(np.diag(n0))) == 0


def test_subpixel_gradient_and_linesearch_match_central_differences():
    o, p, offs, frac = _problem(seed=5)
    iobs = oracle.simulate_intensity(o, p, offs, frac=frac) * 1.05
    o0, p0 = o * np.exp(0.1j), p * 0.95
    g_o, g_p, _ = oracle.ml_grad(o0, p0, offs, iobs, None, frac=frac)
    rng = np.random.default_rng(9)
    for x0, g, f in ((o0, g_o, lambda x: oracle.llk(x, p0, offs, iobs, None, frac=frac)[0]),
                     (p0, g_p, lambda x: oracle.llk(o0, x, offs, iobs, None, frac=frac)[0])):
        h = 1e-4 * np.sqrt((abs(x0) ** 2).mean())
        for i in rng.choice(np.flatnonzero(abs(g) > 0.05 * abs(g).max()), 8, replace=False):
            e = np.zeros(x0.shape, complex)
            e.flat[i] = h
            fd = complex((f(x0 + e) - f(x0 - e)) / (2 * h), (f(x0 + 1j * e) - f(x0 - 1j * e)) / (2 * h))
            assert abs(g.flat[i] - fd) <= 1e-6 * abs(fd), (i, g.flat[i], fd)
    d_o, d_p = crandn(*o.shape, rng=rng) * 1e-2, crandn(*p.shape, rng=rng) * 1e-2
    l1, l2 = oracle.linesearch_coefs(o0, p0, d_o, d_p, offs, iobs, None, frac=frac)
    f = lambda gm: oracle.llk(o0 + gm * d_o, p0 + gm * d_p, offs, iobs, None, frac=frac)[0]
    np.testing.assert_allclose(l1, (f(1e-3) - f(-1e-3)) / 2e-3, rtol=1e-6)
    np.testing.assert_allclose(l2, (f(1e-3) - 2 * f(0.0) + f(-1e-3)) / 1e-6, rtol=1e-4)


def _smooth_object(shape, seed=2):
    rng = np.random.default_rng(seed)
    yy, xx = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), indexing="ij")
    ph = np.zeros(shape)
    for _ in range(6):
        ky, kx = rng.uniform(-0.35, 0.35, 2)
        ph += rng.uniform(0.2, 0.5) * np.cos(ky * yy + kx * xx + rng.uniform(0, 6.3))
    return (0.9 + 0.05 * np.cos(0.2 * yy)) * np.exp(1j * ph)


def test_position_shifts_recover_a_subpixel_displacement_with_subpixel_windows():
    o = _smooth_object((48, 48))
    p = crandn(1, 16, 16, rng=np.random.default_rng(4)) * 0 + 1.0
    p = p * np.exp(-((np.arange(16) - 7.5) ** 2)[None, :, None] / 40 - ((np.arange(16) - 7.5) ** 2)[None, None, :] / 40)
    t = np.array([[10.3, 12.6], [20.75, 8.2], [15.5, 25.45]])
    d = np.array([[0.12, -0.08], [-0.1, 0.05], [0.07, 0.11]])
    offs, frac = np.floor(t).astype(np.int32), t - np.floor(t)
    offs_d, frac_d = np.floor(t + d).astype(np.int32), (t + d) - np.floor(t + d)
    psi = oracle.exit_waves(o, p, offs_d, frac_d)            # the frames were taken at t + d
    sh, e = oracle.position_shifts(o, p, psi, offs, frac)
    np.testing.assert_allclose(sh, d, atol=0.02)
    assert (e > 0).all()


def test_ml_position_shifts_agree_with_the_ap_projection_near_the_fit():
    """The ML reading takes -1/2 of the back-propagated gradient wave as the
    exit-wave change; near the fit it equals the AP correction to first
    order, so the shifts agree with those of the AP projection (each is a
    partial step toward the displacement; the iterations converge), and they
    vanish at the positions the data were taken at."""
    o = _smooth_object((48, 48), seed=6)
    yy, xx = np.meshgrid(np.arange(16) - 7.5, np.arange(16) - 7.5, indexing="ij")
    p = (30.0 * np.exp(-(yy ** 2 + xx ** 2) / 30))[None].astype(complex)
    t = np.array([[10.3, 12.6], [20.75, 8.2], [15.5, 25.45], [12.2, 20.1]])
    d = 0.2 * np.array([[0.15, -0.1], [-0.12, 0.08], [0.1, 0.12], [-0.09, -0.14]])
    offs, frac = np.floor(t).astype(np.int32), t - np.floor(t)
    offs_d, frac_d = np.floor(t + d).astype(np.int32), (t + d) - np.floor(t + d)
    iobs = oracle.simulate_intensity(o, p, offs_d, frac=frac_d)
    sh_ml, _ = oracle.ml_position_shifts(o, p, offs, iobs, None, frac=frac)
    psi = oracle.fourier_project(oracle.exit_waves(o, p, offs, frac), iobs, None)
    sh_ap, _ = oracle.position_shifts(o, p, psi, offs, frac)
    assert np.abs(sh_ap).max() > 5e-3
    assert np.abs(sh_ml - sh_ap).max() <= 0.05 * np.abs(sh_ap).max()
    sh0, _ = oracle.ml_position_shifts(o, p, offs_d, iobs, None, frac=frac_d)
    assert np.abs(sh0).max() < 1e-8


def _refinement_problem():
    rng = np.random.default_rng(1)
    o = _smooth_object((64, 64), seed=6)
    yy, xx = np.meshgrid(np.arange(16) - 7.5, np.arange(16) - 7.5, indexing="ij")
    p = (30.0 * np.exp(-(yy ** 2 + xx ** 2) / 30))[None].astype(complex)
    pos_true = np.stack([rng.uniform(-20, 20, 40), rng.uniform(-20, 20, 40)], axis=1)
    offs, frac = oracle.windows_from_positions(pos_true, 16, o.shape)
    iobs = oracle.simulate_intensity(o, p, offs, frac=frac)
    pos0 = pos_true + rng.choice([-0.3, 0.3], size=pos_true.shape)
    return o, p, pos_true, pos0, iobs


def _relative_error(pos, pos_true):
    d = pos - pos_true
    return np.abs(d - d.mean(axis=0)).mean()       # a common shift of all frames is not observable


def test_ap_refinement_with_a_fixed_object_converges_to_subpixel_positions():
    o, p, pos_true, pos0, iobs = _refinement_problem()
    pos = pos0.copy()
    for _ in range(10):
        offs, frac = oracle.windows_from_positions(pos, 16, o.shape)
        psi = oracle.fourier_project(oracle.exit_waves(o, p, offs, frac), iobs, None)
        sh, e = oracle.position_shifts(o, p, psi, offs, frac)
        pos = oracle.update_positions(pos, pos0, sh, e)
    assert _relative_error(pos, pos_true) < 0.07 < _relative_error(pos0, pos_true)


def test_ml_refinement_with_object_and_probe_updates_converges():
    o, p, pos_true, pos0, iobs = _refinement_problem()
    pos, x_o, x_p, st = pos0.copy(), o.copy(), p.copy(), oracle.CGState()
    for _ in range(12):
        offs, frac = oracle.windows_from_positions(pos, 16, o.shape)
        sh, e = oracle.ml_position_shifts(x_o, x_p, offs, iobs, None, frac=frac)
        x_o, x_p = oracle.ml_cycle(x_o, x_p, st, offs, iobs, None, update=oracle.UPDATE_OBJECT | oracle.UPDATE_PROBE,
                                   frac=frac)
        pos = oracle.update_positions(pos, pos0, sh, e)
    assert np.abs(pos - pos_true).mean() < 0.15 < np.abs(pos0 - pos_true).mean()

"""Pins of the FP64 oracle against facts fixed outside the oracle itself.

Each test checks one oracle function against mathematics that does not go
through that function: explicit DFT sums, Parseval, idempotence, textbook
least squares (numpy.linalg.lstsq on the dense linear model), the scipy
Poisson log-pmf, finite differences and hand-worked scalar cases stored in
tests/golden.  A plausible mistake in the oracle (dropped term, wrong sign,
wrong index, transposed operand) breaks at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(1234)


def crandn(*shape, rng=RNG):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def tiny_problem(n=8, k=2, j=5, obj=(16, 16), seed=7, mask=True, noiseless=True):
    """A small self-consistent problem: truth, offsets, Iobs, mask."""
    rng = np.random.default_rng(seed)
    o = (0.8 + 0.2 * rng.random(obj)) * np.exp(1j * rng.uniform(-1, 1, obj))
    p = crandn(k, n, n, rng=rng) * 3.0
    offs = np.stack([rng.integers(0, obj[0] - n + 1, j),
                     rng.integers(0, obj[1] - n + 1, j)], axis=1).astype(np.int32)
    inten = oracle.simulate_intensity(o, p, offs)
    iobs = inten if noiseless else rng.poisson(inten).astype(np.float64)
    m = None
    if mask:
        m = np.zeros((n, n), dtype=np.uint8)
        m[:, 2] = 1
        m[5, :] = 1
    return o, p, offs, iobs, m


# ----------------------------------------------------------------------------
# FFT: explicit DFT sums, closed forms, Parseval
# ----------------------------------------------------------------------------

def brute_dft2(x, sign):
    n0, n1 = x.shape
    out = np.zeros_like(x, dtype=np.complex128)
    for u in range(n0):
        for v in range(n1):
            acc = 0j
            for y in range(n0):
                for xx in range(n1):
                    acc += x[y, xx] * complex(math.cos(2 * math.pi * (u * y / n0 + v * xx / n1)),
                                              sign * math.sin(2 * math.pi * (u * y / n0 + v * xx / n1)))
            out[u, v] = acc / math.sqrt(n0 * n1)
    return out


@pytest.mark.parametrize("n", [1, 2, 4, 8])
def test_fft_matches_explicit_dft_sum(n):
    x = crandn(n, n)
    np.testing.assert_allclose(oracle.fft2(x), brute_dft2(x, -1.0), rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.ifft2(x), brute_dft2(x, +1.0), rtol=0, atol=1e-12)


def test_fft_delta_and_plane_wave():
    n = 16
    d = np.zeros((n, n), complex)
    d[0, 0] = 1.0
    np.testing.assert_allclose(oracle.fft2(d), np.full((n, n), 1.0 / n), atol=1e-15)
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    u, v = 3, 5
    wave = np.exp(2j * np.pi * (u * y + v * x) / n)       # positive frequency
    f = oracle.fft2(wave)
    expect = np.zeros((n, n), complex)
    expect[u, v] = n                                       # sum/N with unitary norm
    np.testing.assert_allclose(f, expect, atol=1e-12)


def test_fft_parseval_and_roundtrip():
    x = crandn(3, 2, 32, 32)
    f = oracle.fft2(x)
    np.testing.assert_allclose((abs(f) ** 2).sum(axis=(-1, -2)), (abs(x) ** 2).sum(axis=(-1, -2)), rtol=1e-13)
    np.testing.assert_allclose(oracle.ifft2(f), x, atol=1e-13)


# ----------------------------------------------------------------------------
# Positions, offsets and views: integer arithmetic, exact
# ----------------------------------------------------------------------------

def test_offsets_round_half_up_and_bounds():
    # centre of a 64x64 object is 32.0; N = 8 => o = floor(32 + p + 0.5) - 4
    pos = np.array([[0.0, 0.0], [0.5, -0.5], [1.5, -1.5], [2.49999, -2.5],
                    [-0.50000001, 0.49999999]])
    o = oracle.offsets_from_positions(pos, 8, (64, 64))
    assert o.dtype == np.int32
    assert o.tolist() == [[28, 28], [29, 28], [30, 27], [30, 26], [27, 28]]
    with pytest.raises(ValueError):
        oracle.offsets_from_positions(np.array([[29.0, 0.0]]), 8, (64, 64))
    with pytest.raises(ValueError):
        oracle.offsets_from_positions(np.array([[0.0, -28.6]]), 8, (64, 64))
    # the extreme in-bounds windows are accepted
    o = oracle.offsets_from_positions(np.array([[-28.0, 28.0]]), 8, (64, 64))
    assert o.tolist() == [[0, 56]]


def test_views_pick_the_right_pixels():
    ny, nx, n = 20, 24, 4
    obj = np.arange(ny * nx, dtype=np.float64).reshape(ny, nx).astype(complex)
    offs = np.array([[0, 0], [3, 7], [16, 20]], dtype=np.int32)
    v = oracle.views(obj, offs, n)
    for j, (oy, ox) in enumerate(offs):
        for y in range(n):
            for x in range(n):
                assert v[j, y, x] == (oy + y) * nx + (ox + x)
    probe = np.stack([np.full((n, n), 2.0 + 0j), np.full((n, n), 1j)])
    phi = oracle.exit_waves(obj, probe, offs)
    assert phi.shape == (3, 2, n, n)
    np.testing.assert_array_equal(phi[1, 0], 2.0 * v[1])
    np.testing.assert_array_equal(phi[2, 1], 1j * v[2])


# ----------------------------------------------------------------------------
# Modulus projection
# ----------------------------------------------------------------------------

def test_modulus_projection_properties():
    j, k, n = 4, 3, 16
    ph = crandn(j, k, n, n)
    iobs = RNG.random((j, n, n)) * 10
    iobs[0, 0, 0] = 0.0
    mask = np.zeros((n, n), np.uint8)
    mask[3, :] = 1
    out = oracle.project_modulus(ph, iobs, mask)
    good = mask == 0
    inten = (abs(out) ** 2).sum(axis=1)
    np.testing.assert_allclose(inten[:, good], iobs[:, good], rtol=1e-12, atol=1e-14)
    # bad pixels pass through unchanged, bit for bit
    np.testing.assert_array_equal(out[:, :, ~good], ph[:, :, ~good])
    # phases and relative mode amplitudes are kept: out = s * ph with real s >= 0
    ratio = out[:, :, good] / ph[:, :, good]
    np.testing.assert_allclose(ratio.imag, 0, atol=1e-12)
    assert (ratio.real >= 0).all()
    np.testing.assert_allclose(ratio[:, 0], ratio[:, 1], rtol=1e-12)
    # idempotent
    np.testing.assert_allclose(oracle.project_modulus(out, iobs, mask), out, rtol=1e-12, atol=1e-14)
    # zero field stays zero (no NaN), zero counts give zero field
    z = oracle.project_modulus(np.zeros_like(ph), iobs, mask)
    assert np.isfinite(z).all() and (z == 0).all()
    assert (out[0, :, 0, 0] == 0).all()


def test_fourier_project_all_bad_is_identity():
    psi = crandn(2, 2, 8, 8)
    mask = np.ones((8, 8), np.uint8)
    np.testing.assert_allclose(oracle.fourier_project(psi, np.ones((2, 8, 8)), mask), psi, atol=1e-13)


# ----------------------------------------------------------------------------
# Overlap update = least-squares solution of the linear exit-wave model
# ----------------------------------------------------------------------------

def dense_object_operator(probe, offs, obj_shape):
    """Matrix A with (A o)[j,k,y,x] = P_k[y,x] o[oy+y, ox+x]."""
    k, n, _ = probe.shape
    ny, nx = obj_shape
    a = np.zeros((len(offs) * k * n * n, ny * nx), complex)
    row = 0
    for oy, ox in offs:
        for kk in range(k):
            for y in range(n):
                for x in range(n):
                    a[row, (oy + y) * nx + (ox + x)] = probe[kk, y, x]
                    row += 1
    return a


def dense_probe_operator(obj, offs, k, n):
    """Matrix B with (B p)[j,k,y,x] = O[oy+y, ox+x] p[k,y,x]."""
    b = np.zeros((len(offs) * k * n * n, k * n * n), complex)
    row = 0
    for oy, ox in offs:
        for kk in range(k):
            for y in range(n):
                for x in range(n):
                    b[row, (kk * n + y) * n + x] = obj[oy + y, ox + x]
                    row += 1
    return b


def test_object_update_is_least_squares():
    n, k, ny, nx = 4, 2, 9, 10
    offs = np.array([[0, 0], [2, 3], [5, 6], [4, 1]], np.int32)
    probe = crandn(k, n, n)
    obj0 = crandn(ny, nx)
    psi = crandn(len(offs), k, n, n)
    o, p = oracle.overlap_update(obj0, probe, psi, offs, update=oracle.UPDATE_OBJECT,
                                 inertia_obj=0.0)
    a = dense_object_operator(probe, offs, (ny, nx))
    cols = np.abs(a).sum(axis=0) > 0            # illuminated pixels only
    sol, *_ = np.linalg.lstsq(a[:, cols], psi.reshape(-1), rcond=None)
    np.testing.assert_allclose(o.reshape(-1)[cols], sol, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(p, probe)     # probe untouched


def test_probe_update_is_least_squares():
    n, k, ny, nx = 4, 2, 9, 10
    offs = np.array([[0, 0], [2, 3], [5, 6]], np.int32)
    obj = crandn(ny, nx)
    probe0 = crandn(k, n, n)
    psi = crandn(len(offs), k, n, n)
    o, p = oracle.overlap_update(obj, probe0, psi, offs, update=oracle.UPDATE_PROBE,
                                 inertia_probe=0.0)
    b = dense_probe_operator(obj, offs, k, n)
    sol, *_ = np.linalg.lstsq(b, psi.reshape(-1), rcond=None)
    np.testing.assert_allclose(p.reshape(-1), sol, rtol=1e-10, atol=1e-12)
    np.testing.assert_array_equal(o, obj)


def test_update_order_and_inertia_closed_form():
    # One frame, constant probe c: O_new = (conj(c) psi + a O)/( |c|^2 + a ),
    # a = delta * |c|^2 (max of denO); the probe then uses the NEW object.
    n = 4
    c = 1.5 - 0.5j
    obj = crandn(6, 6)
    probe = np.full((1, n, n), c)
    offs = np.array([[1, 2]], np.int32)
    psi = crandn(1, 1, n, n)
    d = 0.25
    o, p = oracle.overlap_update(obj, probe, psi, offs, inertia_obj=d, inertia_probe=d)
    a = d * abs(c) ** 2
    win_new = (np.conj(c) * psi[0, 0] + a * obj[1:5, 2:6]) / (abs(c) ** 2 + a)
    np.testing.assert_allclose(o[1:5, 2:6], win_new, rtol=1e-13)
    untouched = np.ones((6, 6), bool)
    untouched[1:5, 2:6] = False
    np.testing.assert_allclose(o[untouched], obj[untouched], rtol=1e-15)
    den_p = abs(win_new) ** 2
    ap = d * den_p.max()
    np.testing.assert_allclose(p[0], (np.conj(win_new) * psi[0, 0] + ap * c) / (den_p + ap), rtol=1e-12)


def test_update_resolves_the_scale_ambiguity():
    # Exit waves that are exactly c * (O P): the object absorbs c, the probe
    # then stays put, so the product matches the exit waves (no overshoot).
    n = 4
    obj = crandn(8, 8)
    probe = crandn(2, n, n)
    offs = np.array([[0, 0], [2, 3], [4, 1], [3, 4]], np.int32)
    c = 1.7 * np.exp(0.4j)
    psi = c * oracle.exit_waves(obj, probe, offs)
    o, p = oracle.overlap_update(obj, probe, psi, offs, inertia_obj=0.0, inertia_probe=0.0)
    np.testing.assert_allclose(oracle.exit_waves(o, p, offs), psi, rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------------------
# AP / DM
# ----------------------------------------------------------------------------

def test_truth_is_fixed_point_of_ap_and_dm():
    o, p, offs, iobs, m = tiny_problem()
    o1, p1 = oracle.ap_cycle(o, p, offs, iobs, m)
    assert np.abs(o1 - o).max() < 1e-12 * np.abs(o).max()
    assert np.abs(p1 - p).max() < 1e-12 * np.abs(p).max()
    psi = oracle.psi_init(o, p, offs)
    o2, p2, psi2 = oracle.dm_cycle(o, p, psi, offs, iobs, m)
    assert np.abs(psi2 - psi).max() < 1e-12 * np.abs(psi).max()
    assert np.abs(o2 - o).max() < 1e-12 * np.abs(o).max()
    assert np.abs(p2 - p).max() < 1e-12 * np.abs(p).max()


def test_first_dm_cycle_equals_ap():
    o, p, offs, iobs, m = tiny_problem(noiseless=False)
    o0 = o * np.exp(0.3j)            # off the truth
    p0 = p * 1.1
    psi0 = oracle.psi_init(o0, p0, offs)
    o_ap, p_ap = oracle.ap_cycle(o0, p0, offs, iobs, m)
    o_dm, p_dm, psi1 = oracle.dm_cycle(o0, p0, psi0, offs, iobs, m)
    np.testing.assert_allclose(o_dm, o_ap, atol=1e-12)
    np.testing.assert_allclose(p_dm, p_ap, atol=1e-12)
    np.testing.assert_allclose(psi1, oracle.fourier_project(oracle.exit_waves(o0, p0, offs), iobs, m), atol=1e-12)


def test_dm_with_no_fourier_constraint_returns_views():
    o, p, offs, iobs, _ = tiny_problem()
    psi = crandn(len(offs), p.shape[0], 8, 8)
    allbad = np.ones((8, 8), np.uint8)
    _, _, psi1 = oracle.dm_cycle(o, p, psi, offs, iobs, allbad)
    np.testing.assert_allclose(psi1, oracle.exit_waves(o, p, offs), atol=1e-12)


def test_golden_scalar_cases():
    """Hand-worked 1x1-frame cases (the DFT of one pixel is the identity)."""
    with open(os.path.join(GOLDEN, "scalar_cases.json")) as f:
        cases = json.load(f)
    for c in cases["dm"]:
        o = np.array([[complex(*c["obj"])]])
        p = np.array([[[complex(*c["probe"])]]])
        psi = np.array([[[[complex(*c["psi"])]]]])
        offs = np.zeros((1, 2), np.int32)
        _, _, psi1 = oracle.dm_cycle(o, p, psi, offs, np.array([[[c["iobs"]]]]), None)
        assert abs(psi1[0, 0, 0, 0] - complex(*c["psi_new"])) < 1e-12, c
    for c in cases["llk"]:
        assert abs(oracle.llk_terms(np.array(c["icalc"]), np.array(c["iobs"])) - c["term"]) < 1e-12, c
    for c in cases["update"]:
        o = np.array([[complex(*c["obj"])]])
        p = np.array([[[complex(*c["probe"])]]])
        psi = np.array([[[[complex(*c["psi"])]]]])
        offs = np.zeros((1, 2), np.int32)
        o1, p1 = oracle.overlap_update(o, p, psi, offs, inertia_obj=c["delta"], inertia_probe=c["delta"])
        assert abs(o1[0, 0] - complex(*c["obj_new"])) < 1e-12, c
        assert abs(p1[0, 0, 0] - complex(*c["probe_new"])) < 1e-12, c


# ----------------------------------------------------------------------------
# Poisson LLK
# ----------------------------------------------------------------------------

def test_llk_equals_poisson_logpmf_difference():
    rng = np.random.default_rng(5)
    icalc = rng.uniform(0.1, 50.0, 500)
    iobs = rng.poisson(icalc * rng.uniform(0.5, 1.5, 500)).astype(np.float64)
    t = oracle.llk_terms(icalc, iobs)
    ref = scipy.stats.poisson.logpmf(iobs, iobs) - scipy.stats.poisson.logpmf(iobs, icalc)
    np.testing.assert_allclose(t, ref, rtol=1e-10, atol=1e-10)
    assert np.all(oracle.llk_terms(iobs + 1.0, iobs + 1.0) == 0.0)


def test_gaussian_and_euclidean_llk_are_normal_logpdf_differences():
    # Gaussian: counts ~ N(I, Iobs + 1); Euclidean: amplitudes ~ N(sqrt(I), 1/4)
    rng = np.random.default_rng(9)
    icalc = rng.uniform(0.1, 50.0, 400)
    iobs = rng.poisson(icalc * rng.uniform(0.5, 1.5, 400)).astype(np.float64)
    sd = np.sqrt(iobs + 1.0)
    ref_g = scipy.stats.norm.logpdf(iobs, iobs, sd) - scipy.stats.norm.logpdf(iobs, icalc, sd)
    np.testing.assert_allclose(oracle.llk_model_terms(icalc, iobs, "gaussian"), ref_g, rtol=1e-10, atol=1e-10)
    a_obs = np.sqrt(iobs)
    ref_e = scipy.stats.norm.logpdf(a_obs, a_obs, 0.5) - scipy.stats.norm.logpdf(a_obs, np.sqrt(icalc), 0.5)
    np.testing.assert_allclose(oracle.llk_model_terms(icalc, iobs, "euclidean"), ref_e, rtol=1e-10, atol=1e-10)
    np.testing.assert_array_equal(oracle.llk_model_terms(icalc, iobs, "poisson"), oracle.llk_terms(icalc, iobs))
    # hand values at I = 4, Iobs = 9
    assert oracle.llk_model_terms(4.0, 9.0, "gaussian") == 25.0 / 20.0
    assert oracle.llk_model_terms(4.0, 9.0, "euclidean") == 2.0
    with pytest.raises(ValueError):
        oracle.llk_model_terms(4.0, 9.0, "cauchy")


def test_noise_models_agree_to_second_order_near_the_fit():
    iobs = np.array([1e4, 3e4, 1e5])
    for d in (1e-3, -2e-3):
        target = iobs * d * d / 2.0
        for model in oracle.LLK_MODELS:
            t = oracle.llk_model_terms(iobs * (1.0 + d), iobs, model)
            np.testing.assert_allclose(t, target, rtol=3e-3)


def test_llk_sum_excludes_masked_pixels_and_is_zero_at_truth():
    o, p, offs, iobs, m = tiny_problem()
    s, nobs = oracle.llk(o, p, offs, iobs, m)
    for model in oracle.LLK_MODELS:
        sm, nm = oracle.llk(o, p, offs, iobs, m, model=model)
        assert nm == nobs and abs(sm) < 1e-9 * max(1.0, float(np.abs(iobs).sum()))
    assert nobs == len(offs) * int((m == 0).sum())
    assert abs(s) < 1e-9 * iobs.sum()
    iobs2 = iobs.copy()
    iobs2[:, m != 0] = 1e9            # garbage under the mask changes nothing
    s2, _ = oracle.llk(o, p, offs, iobs2, m)
    assert s2 == s
    iobs3 = iobs.copy()
    iobs3[0, 0, 0] += 5.0             # an unmasked pixel does count
    s3, _ = oracle.llk(o, p, offs, iobs3, m)
    assert s3 > s


# ----------------------------------------------------------------------------
# Gradient and line search: finite differences in FP64
# ----------------------------------------------------------------------------

def _fd_check(fun, x, g, idx, h):
    for i in idx:
        e = np.zeros_like(x)
        e.flat[i] = h
        re = (fun(x + e) - fun(x - e)) / (2 * h)
        im = (fun(x + 1j * e) - fun(x - 1j * e)) / (2 * h)
        np.testing.assert_allclose(g.flat[i].real, re, rtol=2e-5, atol=1e-6 * abs(g).max())
        np.testing.assert_allclose(g.flat[i].imag, im, rtol=2e-5, atol=1e-6 * abs(g).max())


def test_gradient_matches_central_differences():
    o, p, offs, iobs, m = tiny_problem(noiseless=False, seed=11)
    o0 = o * np.exp(0.2j * np.cos(np.arange(o.size).reshape(o.shape)))
    p0 = p * 1.05
    g_o, g_p, _ = oracle.ml_grad(o0, p0, offs, iobs, m)
    rng = np.random.default_rng(3)
    lo = lambda x: oracle.llk(x, p0, offs, iobs, m)[0]
    lp = lambda x: oracle.llk(o0, x, offs, iobs, m)[0]
    illum = np.flatnonzero(abs(g_o) > 0)
    _fd_check(lo, o0, g_o, rng.choice(illum, 8, replace=False), 1e-3 * np.sqrt((abs(o0) ** 2).mean()))
    _fd_check(lp, p0, g_p, rng.choice(p0.size, 8, replace=False), 1e-3 * np.sqrt((abs(p0) ** 2).mean()))


def test_gradient_vanishes_at_truth():
    o, p, offs, iobs, m = tiny_problem(seed=13)
    g_o, g_p, _ = oracle.ml_grad(o, p, offs, iobs, m)
    g2_o, g2_p, _ = oracle.ml_grad(o * 1.01, p, offs, iobs, m)
    assert np.linalg.norm(g_o) < 1e-10 * np.linalg.norm(g2_o)
    assert np.linalg.norm(g_p) < 1e-10 * np.linalg.norm(g2_p)


def test_linesearch_coefs_match_exact_llk_along_the_line():
    o, p, offs, iobs, m = tiny_problem(noiseless=False, seed=17)
    o0, p0 = o * np.exp(0.1j), p * 0.97
    rng = np.random.default_rng(4)
    d_o = crandn(*o.shape, rng=rng) * 1e-2
    d_p = crandn(*p.shape, rng=rng) * 1e-2
    l1, l2 = oracle.linesearch_coefs(o0, p0, d_o, d_p, offs, iobs, m)
    f = lambda g: oracle.llk(o0 + g * d_o, p0 + g * d_p, offs, iobs, m)[0]
    h = 1e-3
    np.testing.assert_allclose(l1, (f(h) - f(-h)) / (2 * h), rtol=1e-6)
    np.testing.assert_allclose(l2, (f(h) - 2 * f(0) + f(-h)) / h ** 2, rtol=1e-4)
    # L'(0) is also the directional derivative <g, d> = Re sum conj(g) d
    g_o, g_p, _ = oracle.ml_grad(o0, p0, offs, iobs, m)
    np.testing.assert_allclose(l1, np.vdot(g_o, d_o).real + np.vdot(g_p, d_p).real, rtol=1e-10)


def test_cg_decreases_llk_and_first_step_is_preconditioned_descent():
    o, p, offs, iobs, m = tiny_problem(noiseless=False, seed=19, j=8)
    o0, p0 = o * np.exp(0.3j * np.sin(np.arange(o.size).reshape(o.shape) / 7)), p * 0.9
    st = oracle.CGState()
    x_o, x_p = o0, p0
    upd = oracle.UPDATE_OBJECT | oracle.UPDATE_PROBE
    for _ in range(6):
        x_o, x_p = oracle.ml_cycle(x_o, x_p, st, offs, iobs, m, update=upd)
    hist = st.history
    assert hist[-1] < hist[0]
    # first step: d = -(g_O, s g_P) with s = max denO / max denP
    st2 = oracle.CGState()
    oracle.ml_cycle(o0, p0, st2, offs, iobs, m, update=upd)
    g_o, g_p, _ = oracle.ml_grad(o0, p0, offs, iobs, m)
    den_o, den_p = oracle.overlap_denominators(o0, p0, offs)
    np.testing.assert_allclose(st2.d_obj, -g_o, atol=1e-12 * abs(g_o).max())
    np.testing.assert_allclose(st2.d_probe, -(den_o.max() / den_p.max()) * g_p, atol=1e-12 * abs(g_p).max())


def test_denominators_from_sums():
    o, p, offs, iobs, m = tiny_problem()
    psi = crandn(len(offs), p.shape[0], 8, 8)
    _, den_o, _, den_p = oracle.overlap_sums(psi, o, p, offs)
    d_o, d_p = oracle.overlap_denominators(o, p, offs)
    np.testing.assert_allclose(d_o, den_o, rtol=1e-14)
    np.testing.assert_allclose(d_p, den_p, rtol=1e-14)
    # denO counts every covering frame: with P = 1 it is the coverage count
    d_o1, _ = oracle.overlap_denominators(o, np.ones((1, 8, 8)), offs)
    cover = np.zeros(o.shape)
    for oy, ox in offs:
        cover[oy:oy + 8, ox:ox + 8] += 1
    np.testing.assert_array_equal(d_o1, cover)


# ----------------------------------------------------------------------------
# Synthetic generator sanity (inputs, not the method)
# ----------------------------------------------------------------------------

def test_generator_shapes_and_scaling():
    w = synth.workload("ap64")
    o = synth.object_truth(w.obj_shape, w.seed)
    assert o.shape == w.obj_shape
    assert 0.8 <= abs(o).min() and abs(o).max() <= 1.0
    p = synth.probe_modes(w.n, 3, w.seed)
    np.testing.assert_allclose((abs(p) ** 2).sum(axis=(1, 2)), [0.7, 0.2, 0.1], rtol=1e-12)
    assert abs(np.vdot(p[0], p[1])) < 1e-12
    pos = synth.spiral_positions(w.n_frames, w.step)
    offs = oracle.offsets_from_positions(pos, w.n, w.obj_shape)
    sc = synth.probe_photon_scale(o, p, offs, 1e6)
    inten = oracle.simulate_intensity(o, p * sc, offs)
    np.testing.assert_allclose(inten.sum(axis=(1, 2)).mean(), 1e6, rtol=1e-10)
    m = synth.gap_mask(256, 0.02, 1)
    assert abs(m.mean() - 6 * 256 / 256 ** 2) < 1e-12


def test_dm_stays_bounded_over_many_cycles():
    """With the object-then-probe update the DM iteration on noisy data stays
    bounded and does not lose likelihood (it diverged by orders of magnitude
    when both factors were updated from the same old pair)."""
    import cases
    wl = cases.small("dm256", n=64, k=2, j=80, obj=(256, 256), step=6.0, mask_frac=0.03)
    pb = cases.make_problem(wl, start="ml")
    o, p = pb.obj0, pb.probe0
    psi = oracle.psi_init(o, p, pb.offsets)
    l0 = oracle.llk(o, p, pb.offsets, pb.iobs, pb.mask)[0]
    for _ in range(30):
        o, p, psi = oracle.dm_cycle(o, p, psi, pb.offsets, pb.iobs, pb.mask)
    assert np.abs(o).max() < 3.0
    assert oracle.llk(o, p, pb.offsets, pb.iobs, pb.mask)[0] < 2 * l0


# ----------------------------------------------------------------------------
# Incoherent background
# ----------------------------------------------------------------------------

def _background(n, seed=4):
    rng = np.random.default_rng(seed)
    return 0.5 + rng.random((n, n))


def test_zero_background_changes_nothing():
    o, p, offs, iobs, m = tiny_problem(noiseless=False, seed=12)
    o0, p0 = o * 1.01, p * 0.97
    z = np.zeros(p.shape[1:])
    upd = oracle.UPDATE_OBJECT | oracle.UPDATE_PROBE
    a = oracle.ap_cycle(o0, p0, offs, iobs, m, upd)
    b = oracle.ap_cycle(o0, p0, offs, iobs, m, upd | oracle.UPDATE_BACKGROUND, bg=z)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])
    assert not b[2].any()
    psi = oracle.psi_init(o0, p0, offs)
    for x, y in zip(oracle.dm_cycle(o0, p0, psi, offs, iobs, m), oracle.dm_cycle(o0, p0, psi, offs, iobs, m, bg=z)):
        np.testing.assert_array_equal(x, y)
    assert oracle.llk(o0, p0, offs, iobs, m) == oracle.llk(o0, p0, offs, iobs, m, bg=z)
    for x, y in zip(oracle.ml_grad(o0, p0, offs, iobs, m), oracle.ml_grad(o0, p0, offs, iobs, m, bg=z)):
        np.testing.assert_array_equal(x, y)


def test_truth_with_background_is_a_fixed_point():
    o, p, offs, _, m = tiny_problem(seed=13)
    bg = _background(p.shape[-1])
    iobs = oracle.simulate_intensity(o, p, offs, bg=bg)
    all3 = oracle.UPDATE_OBJECT | oracle.UPDATE_PROBE | oracle.UPDATE_BACKGROUND
    o1, p1, b1 = oracle.ap_cycle(o, p, offs, iobs, m, all3, bg=bg)
    assert np.abs(o1 - o).max() < 1e-12 and np.abs(p1 - p).max() < 1e-12
    assert np.abs(b1 - bg).max() < 1e-12
    psi = oracle.psi_init(o, p, offs)
    o2, p2, _ = oracle.dm_cycle(o, p, psi, offs, iobs, m, bg=bg)
    assert np.abs(o2 - o).max() < 1e-12 and np.abs(p2 - p).max() < 1e-12
    assert abs(oracle.llk(o, p, offs, iobs, m, bg=bg)[0]) < 1e-9 * iobs.sum()
    g_o, g_p, _ = oracle.ml_grad(o, p, offs, iobs, m, bg=bg)
    assert np.abs(g_o).max() < 1e-9 and np.abs(g_p).max() < 1e-9
    # without the background in the model the truth is no longer a fit
    assert oracle.llk(o, p, offs, iobs, m)[0] > 1.0


def test_background_ap_cycle_scalar_case():
    # one pixel, two frames at the same place, O = P = 1, background 2:
    # I = 1 + 2 = 3 for both; Iobs = 6 and 3 give s^2 = 2 and 1, so the new
    # background is 2 * (2 + 1) / 2 = 3, and the object sum is sqrt(2) + 1
    # over a denominator 2 (inertia 1e-2 * 2 on both)
    o = np.ones((1, 1), complex)
    p = np.ones((1, 1, 1), complex)
    offs = np.zeros((2, 2), np.int32)
    iobs = np.array([6.0, 3.0]).reshape(2, 1, 1)
    o1, p1, b1 = oracle.ap_cycle(o, p, offs, iobs, None, oracle.UPDATE_OBJECT | oracle.UPDATE_BACKGROUND,
                                 bg=np.full((1, 1), 2.0))
    assert b1[0, 0] == pytest.approx(3.0, rel=1e-15)
    assert o1[0, 0] == pytest.approx((np.sqrt(2.0) + 1.0 + 0.02) / 2.02, rel=1e-15)
    assert p1[0, 0, 0] == 1.0
    with pytest.raises(ValueError):
        oracle.ap_cycle(o, p, offs, iobs, None, oracle.UPDATE_BACKGROUND)


def test_gradient_with_background_matches_central_differences():
    o, p, offs, _, m = tiny_problem(seed=14)
    bg = _background(p.shape[-1], seed=5)
    rng = np.random.default_rng(14)
    iobs = rng.poisson(oracle.simulate_intensity(o, p, offs, bg=bg)).astype(np.float64)
    o0 = o * np.exp(0.2j * np.sin(np.arange(o.size).reshape(o.shape)))
    p0 = p * 0.95
    g_o, g_p, _ = oracle.ml_grad(o0, p0, offs, iobs, m, bg=bg)
    lo = lambda x: oracle.llk(x, p0, offs, iobs, m, bg=bg)[0]
    lp = lambda x: oracle.llk(o0, x, offs, iobs, m, bg=bg)[0]
    illum = np.flatnonzero(abs(g_o) > 0)
    _fd_check(lo, o0, g_o, rng.choice(illum, 8, replace=False), 1e-3 * np.sqrt((abs(o0) ** 2).mean()))
    _fd_check(lp, p0, g_p, rng.choice(p0.size, 8, replace=False), 1e-3 * np.sqrt((abs(p0) ** 2).mean()))
    d_o = o0 * 0.01j
    d_p = p0 * 0.02
    l1, l2 = oracle.linesearch_coefs(o0, p0, d_o, d_p, offs, iobs, m, bg=bg)
    f = lambda g: oracle.llk(o0 + g * d_o, p0 + g * d_p, offs, iobs, m, bg=bg)[0]
    h = 1e-3
    assert l1 == pytest.approx((f(h) - f(-h)) / (2 * h), rel=1e-5)
    assert l2 == pytest.approx((f(h) - 2 * f(0) + f(-h)) / (h * h), rel=1e-3)


# ----------------------------------------------------------------------------
# Position refinement
# ----------------------------------------------------------------------------

def _fourier_shift(a, dy, dx):
    """a(r + d) for a periodic array, by the Fourier shift theorem."""
    ky = np.fft.fftfreq(a.shape[0])[:, None]
    kx = np.fft.fftfreq(a.shape[1])[None, :]
    return np.fft.ifft2(np.fft.fft2(a) * np.exp(2j * np.pi * (ky * dy + kx * dx)))


def test_position_shifts_recover_a_subpixel_displacement():
    # a smooth periodic object: exit waves at r_j + d built by the Fourier
    # shift theorem (not by the gradient) are read back as d to first order
    rng = np.random.default_rng(21)
    ny = nx = 96
    k = np.fft.fftfreq(ny)
    filt = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) * (ny / 6.0) ** 2)

    def field():
        f = np.fft.ifft2(np.fft.fft2(rng.standard_normal((ny, nx))) * filt).real
        return f / f.std()
    # phase of 1 rad rms and 10% amplitude modulation, correlated over ~10 px,
    # so that centred differences are close to the derivative
    o = np.exp(1j * field()) * (1.0 + 0.1 * field())
    n = 32
    y, x = np.mgrid[0:n, 0:n] - n / 2
    p = np.exp(-(x ** 2 + y ** 2) / (2 * 6.0 ** 2))[None].astype(complex)
    offs = np.array([[20, 24], [40, 30], [32, 50]], np.int32)
    d = np.array([[0.15, -0.1], [-0.2, 0.05], [0.0, 0.2]])
    psi = np.zeros((3, 1, n, n), complex)
    for j, ((oy, ox), (dy, dx)) in enumerate(zip(offs, d)):
        psi[j, 0] = p[0] * _fourier_shift(o, dy, dx)[oy:oy + n, ox:ox + n]
    sh, e = oracle.position_shifts(o, p, psi, offs)
    np.testing.assert_allclose(sh, d, atol=0.01)
    assert (e > 0).all()
    # the current views themselves give no shift
    sh0, _ = oracle.position_shifts(o, p, oracle.exit_waves(o, p, offs), offs)
    assert np.abs(sh0).max() < 1e-12


def test_flat_object_gives_no_shift_and_update_rules():
    o = np.full((40, 40), 0.7 + 0.2j)
    p = crandn(2, 8, 8, rng=np.random.default_rng(2))
    offs = np.array([[3, 5], [20, 11]], np.int32)
    psi = oracle.exit_waves(o, p, offs) * 1.3
    sh, e = oracle.position_shifts(o, p, psi, offs)
    assert not sh.any() and not e.any()
    pos0 = np.zeros((4, 2))
    pos = np.array([[0.5, 0.0], [1.9, -1.0], [0.0, 0.0], [-1.5, 0.3]])
    shifts = np.array([[0.2, 0.1], [0.5, 0.0], [1.0, 1.0], [-1.0, 0.2]])
    energy = np.array([1.0, 1.0, 0.01, 1.0])
    new = oracle.update_positions(pos, pos0, shifts, energy, mult=1.0, max_shift=2.0, min_grad=0.1)
    np.testing.assert_allclose(new, [[0.7, 0.1], [2.0, -1.0], [0.0, 0.0], [-2.0, 0.5]])

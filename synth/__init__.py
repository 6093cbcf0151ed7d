"""Seeded synthetic inputs for far- and near-field ptychography workloads.

This module only draws and shapes the *inputs* of a reconstruction: the
ground-truth object, the probe modes, the scan positions, the detector gap
mask and the starting estimates.  It holds none of the reconstruction's
arithmetic (no propagation, no projection, no likelihood).  Both the FP64
oracle and the GPU path consume what it returns; neither is imported here.

The paper's measured workloads (Table 1: 1000 frames of 256x256 with 1 or 3
probe modes; Section 4: 400x400 frames with 3 modes, 6560 positions) are real
beamline datasets that are not available, so every array here stands in for
them with the same shapes and value ranges:

* object: amplitude i.i.d. uniform in [0.8, 1], phase = Gaussian-smoothed
  white noise (sigma 2 px), shifted to zero mean and scaled to 0.5 rad std;
* probe: Gaussian amplitude (FWHM = 20 px per 64 px of frame) times a random
  quadratic phase; extra incoherent modes (Section 4, probe modes) are the
  first mode times the polynomials x, y, xy, orthonormalised and weighted so
  that mode k carries a fixed fraction of the total probe intensity;
* positions: a Fermat spiral (radius step*sqrt(n), golden angle) centred on
  the object, in pixels (float64, (y, x));
* mask: vertical and horizontal 6 px detector-gap bands covering about the
  requested fraction of a frame, generated in detector-centred coordinates
  and returned in FFT order (zero frequency at [0, 0]), 1 = bad pixel.

Near-field workloads (Table 1: 17 frames of 2048x2048, one probe) use a broad
structured illumination instead of the focused spot: a soft-edged aperture
over most of the frame times a smooth random amplitude and phase (a
diffuser), a few scan positions drawn uniformly in a small square, and the
detector in natural pixel order.  Their Fresnel parameter f = pi lambda z /
(N dx)^2 is part of the workload.

All randomness comes from ``numpy.random.SeedSequence`` so that a workload is
reproducible bit for bit from its seed.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np
import scipy.ndimage

__all__ = [
    "Workload", "WORKLOADS", "workload", "make_rng", "object_truth",
    "probe_modes", "spiral_positions", "gap_mask", "start_object",
    "start_probe", "perturb_object", "perturb_probe", "probe_photon_scale",
    "serve_requests", "mode_weights", "poisson_counts",
    "near_field_probe", "random_positions", "fresnel_parameter",
]

BASE_SEED = 20081151


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic ptychography workload (sizes in pixels; far field unless
    geometry is "near")."""

    name: str
    n: int                 # frame (= probe window) side, power of two
    n_modes: int           # incoherent probe modes K
    n_frames: int          # scan positions J
    obj_shape: tuple       # (Ny, Nx)
    step: float            # Fermat spiral step (px)
    photons: float         # mean total photons per frame
    mask_frac: float       # requested fraction of masked detector pixels
    algorithm: str         # "ap", "dm", "ml", "ap+dm"
    cycles: tuple          # cycle counts for the algorithm chain
    seed: int
    geometry: str = "far"  # "far" or "near"
    fresnel: float = 0.0   # near field: f = pi lambda z / (N dx)^2 (both axes)

    def scaled(self, n_frames: int) -> "Workload":
        """Same model with fewer scan positions (parity tests, samples)."""
        return dataclasses.replace(self, n_frames=int(n_frames),
                                   name=f"{self.name}@J{n_frames}")


WORKLOADS = {
    # Plain AP, 64x64 frames, one mode, 100 positions, 10 cycles.
    "ap64": Workload("ap64", 64, 1, 100, (256, 256), 6.0, 1e6, 0.0,
                     "ap", (10,), BASE_SEED + 0),
    # DM, 256x256 frames, 3 modes, 1000 positions, 2% gap mask, 100 cycles.
    "dm256": Workload("dm256", 256, 3, 1000, (1024, 1024), 12.0, 1e8, 0.02,
                      "dm", (100,), BASE_SEED + 1),
    # ML (conjugate gradient), 256x256 frames, 3 modes, 500 positions.
    "ml256": Workload("ml256", 256, 3, 500, (1024, 1024), 12.0, 1e7, 0.02,
                      "ml", (50,), BASE_SEED + 2),
    # Large: 512x512 frames, 4 modes, 4000 positions, 3% mask, 20 AP + 50 DM.
    "apdm512": Workload("apdm512", 512, 4, 4000, (4096, 4096), 24.0, 1e9,
                        0.03, "ap+dm", (20, 50), BASE_SEED + 3),
    # Near field (Table 1): 17 frames of 2048x2048, one probe, positions in a
    # 256 px square, 1e4 photons per pixel, no detector gaps, DM then ML.
    # `step` is the side of the position square.
    "nf2048": Workload("nf2048", 2048, 1, 17, (2368, 2368), 256.0, 1e4 * 2048 ** 2, 0.0,
                       "dm+ml", (400, 100), BASE_SEED + 5, "near", 0.0),
    # The same geometry at 1024x1024 frames (the same Fresnel number per pixel).
    "nf1024": Workload("nf1024", 1024, 1, 17, (1344, 1344), 256.0, 1e4 * 1024 ** 2, 0.0,
                       "dm+ml", (400, 100), BASE_SEED + 6, "near", 0.0),
}

# Fresnel number per pixel, dx^2 / (lambda z), of the near-field workloads.
NEAR_FIELD_NF_PIXEL = 4e-3


def fresnel_parameter(n: int, fresnel_number: float = NEAR_FIELD_NF_PIXEL) -> float:
    """f = pi lambda z / (N dx)^2 = pi / (N^2 N_F) for a Fresnel number per
    pixel N_F = dx^2 / (lambda z)."""
    return math.pi / (n * n * fresnel_number)


for _name in ("nf2048", "nf1024"):
    WORKLOADS[_name] = dataclasses.replace(WORKLOADS[_name], fresnel=fresnel_parameter(WORKLOADS[_name].n))


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def make_rng(seed: int, stream: str) -> np.random.Generator:
    """Independent generator per (seed, stream) so streams never interleave."""
    keys = {"object": 0, "probe": 1, "positions": 2, "noise": 3, "mask": 4,
            "start": 5, "serve": 6, "background": 7}
    ss = np.random.SeedSequence([int(seed), keys[stream]])
    return np.random.Generator(np.random.PCG64(ss))


def object_truth(shape, seed: int, phase_std: float = 0.5,
                 smooth_px: float = 2.0) -> np.ndarray:
    """Ground-truth complex object (complex128)."""
    rng = make_rng(seed, "object")
    ny, nx = shape
    amp = rng.uniform(0.8, 1.0, size=(ny, nx))
    noise = rng.standard_normal((ny, nx))
    ph = scipy.ndimage.gaussian_filter(noise, smooth_px, mode="wrap")
    ph = ph - ph.mean()
    ph = ph * (phase_std / ph.std())
    return amp * np.exp(1j * ph)


def mode_weights(k: int) -> np.ndarray:
    """Fraction of the total probe intensity carried by each mode."""
    table = {1: [1.0], 2: [0.8, 0.2], 3: [0.7, 0.2, 0.1],
             4: [0.7, 0.2, 0.07, 0.03]}
    if k not in table:
        raise ValueError(f"no mode-weight table for {k} modes")
    return np.asarray(table[k], dtype=np.float64)


def _grid(n: int):
    c = np.arange(n, dtype=np.float64) - n / 2.0
    return np.meshgrid(c, c, indexing="ij")   # (y, x)


def probe_modes(n: int, k: int, seed: int) -> np.ndarray:
    """Orthogonal probe modes [K][N][N] (complex128), unit total intensity.

    Mode 0 is a Gaussian spot with a random quadratic (defocus-like) phase;
    modes 1.. are mode 0 times x, y, x*y (in units of the Gaussian sigma),
    Gram-Schmidt orthonormalised, then scaled so that ||P_k||^2 equals the
    mode's intensity fraction.
    """
    rng = make_rng(seed, "probe")
    y, x = _grid(n)
    fwhm = 20.0 * n / 64.0
    sigma = fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))
    r2 = (x * x + y * y) / (n / 2.0) ** 2
    a = rng.uniform(-1.0, 1.0)
    p0 = np.exp(-(x * x + y * y) / (2 * sigma * sigma)) * np.exp(1j * a * math.pi * r2)
    basis = [np.ones_like(x), x / sigma, y / sigma, x * y / sigma ** 2]
    if k > len(basis):
        raise ValueError("at most 4 probe modes are generated")
    modes = []
    for i in range(k):
        v = p0 * basis[i]
        for m in modes:
            v = v - np.vdot(m, v) * m
        v = v / np.sqrt(np.vdot(v, v).real)
        modes.append(v)
    w = mode_weights(k)
    return np.stack([np.sqrt(w[i]) * modes[i] for i in range(k)])


def random_positions(n_frames: int, extent: float, seed: int) -> np.ndarray:
    """Near-field scan: the first position at (0, 0), the others uniform in
    the square [-extent/2, extent/2)^2, (y, x) in pixels."""
    rng = make_rng(seed, "positions")
    pos = rng.uniform(-extent / 2.0, extent / 2.0, size=(n_frames, 2))
    pos[0] = 0.0
    return pos


def near_field_probe(n: int, k: int, seed: int) -> np.ndarray:
    """Near-field illumination modes [K][N][N] (complex128), unit total
    intensity: a square aperture over 90% of the frame with Gaussian-softened
    edges (sigma N/64), times a diffuser: amplitude 1 + 0.3 u and phase
    1.0 v rad, with u, v white noise smoothed over N/128 px and scaled to unit
    peak / unit std.  Extra modes are mode 0 times x, y, xy (in units of N/4),
    orthonormalised and weighted as in `probe_modes`."""
    rng = make_rng(seed, "probe")
    y, x = _grid(n)
    half = 0.45 * n
    ap = ((np.abs(y) <= half) & (np.abs(x) <= half)).astype(np.float64)
    ap = scipy.ndimage.gaussian_filter(ap, n / 64.0, mode="constant")
    sm = max(1.0, n / 128.0)
    u = scipy.ndimage.gaussian_filter(rng.standard_normal((n, n)), sm, mode="wrap")
    v = scipy.ndimage.gaussian_filter(rng.standard_normal((n, n)), sm, mode="wrap")
    u = u / np.abs(u).max()
    v = (v - v.mean()) / v.std()
    p0 = ap * (1.0 + 0.3 * u) * np.exp(1j * v)
    s = n / 4.0
    basis = [np.ones_like(x), x / s, y / s, x * y / s ** 2]
    if k > len(basis):
        raise ValueError("at most 4 probe modes are generated")
    modes = []
    for i in range(k):
        w = p0 * basis[i]
        for m in modes:
            w = w - np.vdot(m, w) * m
        modes.append(w / np.sqrt(np.vdot(w, w).real))
    wt = mode_weights(k)
    return np.stack([np.sqrt(wt[i]) * modes[i] for i in range(k)])


def spiral_positions(n_frames: int, step: float) -> np.ndarray:
    """Fermat spiral scan positions (y, x) in pixels, centred on (0, 0)."""
    i = np.arange(n_frames, dtype=np.float64)
    r = step * np.sqrt(i)
    th = i * math.pi * (3.0 - math.sqrt(5.0))
    return np.stack([r * np.sin(th), r * np.cos(th)], axis=1)


def gap_mask(n: int, frac: float, seed: int, fft_order: bool = True) -> Optional[np.ndarray]:
    """Detector-gap mask u8 [N][N] (1 = bad), or None: in FFT order for the
    far field, in natural order (fft_order False) for the near field."""
    if frac <= 0:
        return None
    rng = make_rng(seed, "mask")
    nb = max(1, int(round(frac * n / 6.0)))
    m = np.zeros((n, n), dtype=np.uint8)
    for b in range(nb):
        start = int(rng.integers(n // 8, n - n // 8 - 6))
        if b % 2 == 0:
            m[:, start:start + 6] = 1     # vertical band
        else:
            m[start:start + 6, :] = 1     # horizontal band
    return np.ascontiguousarray(np.fft.ifftshift(m) if fft_order else m)


def background(n: int, level: float, seed: int) -> np.ndarray:
    """Incoherent background float64 [N][N] in FFT order: a diffuse profile
    1 / (1 + (r / (N/8))^2) about the detector centre times a smooth 0.8-1.2
    random factor, scaled to a mean of `level` photons per pixel."""
    rng = make_rng(seed, "background")
    y, x = np.mgrid[0:n, 0:n] - n // 2
    prof = 1.0 / (1.0 + (np.hypot(y, x) / (n / 8.0)) ** 2)
    noise = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n)
    noise = np.fft.ifft2(np.fft.fft2(noise) * np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) * (n / 4.0) ** 2)).real
    noise = 1.0 + 0.2 * noise / max(np.abs(noise).max(), 1e-12)
    bg = prof * noise
    return np.ascontiguousarray(np.fft.ifftshift(bg * (level / bg.mean())))


def probe_photon_scale(obj: np.ndarray, probe: np.ndarray,
                       offsets: np.ndarray, photons: float) -> float:
    """Scale factor for the probe so that the mean frame holds `photons`.

    The total intensity of a frame equals the real-space energy of its exit
    waves (the propagator is unitary), so the scale is found without any
    propagation: mean over frames of sum_k sum_r |O(r+o_j)|^2 |P_k(r)|^2.
    """
    n = probe.shape[-1]
    pint = (np.abs(probe) ** 2).sum(axis=0)
    o2 = np.abs(obj) ** 2
    tot = 0.0
    for oy, ox in offsets:
        tot += float((o2[oy:oy + n, ox:ox + n] * pint).sum())
    mean = tot / len(offsets)
    return math.sqrt(photons / mean)


def start_object(shape) -> np.ndarray:
    """AP/DM starting object: constant 1."""
    return np.ones(shape, dtype=np.complex128)


def start_probe(probe_true: np.ndarray) -> np.ndarray:
    """AP/DM starting probe: the true probe with an extra mild defocus."""
    n = probe_true.shape[-1]
    y, x = _grid(n)
    r2 = (x * x + y * y) / (n / 2.0) ** 2
    return probe_true * np.exp(1j * 0.5 * r2)[None]


def perturb_object(obj: np.ndarray, seed: int, rad: float = 0.2) -> np.ndarray:
    """ML start: truth times a smooth random phase of `rad` rad std."""
    rng = make_rng(seed, "start")
    noise = scipy.ndimage.gaussian_filter(rng.standard_normal(obj.shape), 4.0,
                                          mode="wrap")
    noise = (noise - noise.mean()) / noise.std() * rad
    return obj * np.exp(1j * noise)


def perturb_probe(probe: np.ndarray, seed: int, amp: float = 0.1) -> np.ndarray:
    """ML start: truth with 10% smooth amplitude noise."""
    rng = make_rng(seed + 7, "start")
    noise = scipy.ndimage.gaussian_filter(
        rng.standard_normal(probe.shape), (0, 3.0, 3.0), mode="wrap")
    noise = noise / noise.std() * amp
    return probe * (1.0 + noise)


def serve_requests(n_requests: int = 64, rate: float = 2.0, seed: int = 0,
                   sizes: Sequence[int] = (128, 256, 512),
                   frames: tuple = (200, 2000), modes: Sequence[int] = (1, 3),
                   min_side: int = 1024):
    """Arrival trace for a served mixed workload.

    Poisson arrivals at `rate` req/s; frame side uniform over `sizes`; scan
    positions uniform in `frames`; probe modes uniform over `modes`.  Objects
    are sized to hold the spiral: side = max(1024, roundup64(2*ceil(r_max) +
    N + 16)), step 12 px, 1e8 photons per frame, 2% gap mask as in the DM
    256x256 workload (`min_side` replaces 1024 for small test traces).
    """
    rng = make_rng(BASE_SEED * 100 + 4 + seed, "serve")
    t = 0.0
    reqs = []
    for i in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        n = int(rng.choice(np.asarray(sizes)))
        j = int(rng.integers(frames[0], frames[1] + 1))
        k = int(rng.choice(np.asarray(modes)))
        step = 12.0
        rmax = step * math.sqrt(max(j - 1, 0))
        side = 2 * int(math.ceil(rmax)) + n + 16
        side = max(min_side, ((side + 63) // 64) * 64)
        wl = Workload(f"req{i}", n, k, j, (side, side), step, 1e8, 0.02,
                      "dm+ml", (30, 20), BASE_SEED * 100 + 4 + 1000 * seed + i)
        reqs.append((t, wl))
    return reqs


def poisson_counts(intensity: np.ndarray, seed: int) -> np.ndarray:
    """Poisson photon counts drawn from given mean intensities (float32).

    Only the random draw lives here; the mean intensities come from a forward
    model computed elsewhere.
    """
    rng = make_rng(seed, "noise")
    lam = np.maximum(np.asarray(intensity, dtype=np.float64), 0.0)
    return rng.poisson(lam).astype(np.float32)

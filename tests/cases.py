"""Seeded test problems shared by the parity tests.

Inputs come from `synth` (truth, positions, mask, start states); offsets and
the noise-free intensities come from the oracle; Poisson draws from `synth`.
Nothing here is produced by the GPU path.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

import oracle
import synth


@dataclasses.dataclass
class Problem:
    wl: synth.Workload
    obj_true: np.ndarray
    probe_true: np.ndarray
    offsets: np.ndarray
    iobs: np.ndarray           # float32 [J][N][N]
    mask: Optional[np.ndarray]
    obj0: np.ndarray
    probe0: np.ndarray
    bg_true: Optional[np.ndarray] = None   # incoherent background in the data
    bg0: Optional[np.ndarray] = None       # its starting estimate
    nf: Optional[float] = None             # near-field Fresnel parameter, None = far field


def make_problem(wl: synth.Workload, start: str = "apdm", noiseless: bool = False,
                 bg_level: float = 0.0) -> Problem:
    near = wl.geometry == "near"
    nf = wl.fresnel if near else None
    obj = synth.object_truth(wl.obj_shape, wl.seed)
    if near:
        probe = synth.near_field_probe(wl.n, wl.n_modes, wl.seed)
        pos = synth.random_positions(wl.n_frames, wl.step, wl.seed)
    else:
        probe = synth.probe_modes(wl.n, wl.n_modes, wl.seed)
        pos = synth.spiral_positions(wl.n_frames, wl.step)
    offs = oracle.offsets_from_positions(pos, wl.n, wl.obj_shape)
    probe = probe * synth.probe_photon_scale(obj, probe, offs, wl.photons)
    bg = synth.background(wl.n, bg_level, wl.seed) if bg_level > 0 else None
    if bg is not None and near:
        bg = np.fft.fftshift(bg)            # detector-centred in natural order
    inten = oracle.simulate_intensity(obj, probe, offs, bg=bg, nf=nf)
    iobs = inten.astype(np.float32) if noiseless else synth.poisson_counts(inten, wl.seed)
    mask = synth.gap_mask(wl.n, wl.mask_frac, wl.seed, fft_order=not near)
    if start == "ml":
        o0 = synth.perturb_object(obj, wl.seed)
        p0 = synth.perturb_probe(probe, wl.seed)
    elif start == "truth":
        o0, p0 = obj.copy(), probe.copy()
    else:
        o0 = synth.start_object(wl.obj_shape)
        p0 = synth.start_probe(probe)
    # everything the GPU sees is complex64 / float32; the oracle runs on the
    # same rounded values promoted to float64
    o0 = o0.astype(np.complex64).astype(np.complex128)
    p0 = p0.astype(np.complex64).astype(np.complex128)
    bg0 = None
    if bg is not None:
        bg0 = (0.7 * bg).astype(np.float32).astype(np.float64)     # 30% low at every start
    return Problem(wl, obj, probe, offs, iobs, mask, o0, p0, bg, bg0, nf)


def small(name: str, n=None, k=None, j=None, obj=None, step=None, mask_frac=None, photons=None, seed_offset=0,
          fresnel=None):
    """A reduced variant of a named workload."""
    wl = synth.workload(name)
    rep = {}
    if n is not None:
        rep["n"] = n
    if k is not None:
        rep["n_modes"] = k
    if j is not None:
        rep["n_frames"] = j
    if obj is not None:
        rep["obj_shape"] = obj
    if step is not None:
        rep["step"] = step
    if mask_frac is not None:
        rep["mask_frac"] = mask_frac
    if photons is not None:
        rep["photons"] = photons
    if fresnel is not None:
        rep["fresnel"] = fresnel
    rep["seed"] = wl.seed + seed_offset
    rep["name"] = f"{name}-small"
    return dataclasses.replace(wl, **rep)


def rel_l2(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))

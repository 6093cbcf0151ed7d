"""Plain FP64 reference for the ptychography hot path (far and near field).

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import this module.  It shares no code,
table or constant generator with the GPU library and imports nothing from it.

Everything is complex128 / float64, uses `numpy.fft` with the unitary
normalisation as the only library primitive, and loops over frames
explicitly.  Each function names the passage of the paper it follows
(Favre-Nicolin et al., "PyNX: high performance computing toolkit for coherent
X-ray imaging based on operators", arXiv 2008.11511).  The paper names the
operators and cites the algorithms but prints no ptychography equations
beyond the exit wave of the ptychography-operator table; where it is silent
the reading taken is stated in the docstring.

Notation: J frames, K probe modes, N x N frames, object Ny x Nx.
  obj     [Ny][Nx]        complex
  probe   [K][N][N]       complex
  offsets [J][2]          int   top-left corner (oy, ox) of each frame's window
  iobs    [J][N][N]       float observed intensity; far field: FFT order (q = 0 at
                          [0, 0]); near field: detector pixels in natural order
  mask    [N][N] or None  uint8, 1 = bad detector pixel (shared by all frames)
  psi     [J][K][N][N]    complex exit waves

The near-field geometry (`nf` arguments: Fresnel parameters, see
`near_field_transfer`) replaces the far-field FT by the unitary near-field
propagation; every other step is unchanged.

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: brute-force DFT sums, Parseval, the paraxial Gaussian beam and the
Talbot self-image for the near-field propagation, idempotence of the modulus
projection, least-squares solutions, fixed points at the truth, the
scipy.stats Poisson log-pmf, and central finite differences.  The CG and DM
*trajectories* over many cycles have no closed form: parity unpinned for the
multi-cycle trajectories beyond each single step's pins.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "fft2", "ifft2", "offsets_from_positions", "views", "exit_waves",
    "calc_intensity", "project_modulus", "fourier_project", "overlap_sums",
    "overlap_denominators", "overlap_update", "ap_cycle", "dm_cycle",
    "psi_init", "llk", "llk_terms", "llk_model_terms", "LLK_MODELS", "ml_grad", "linesearch_coefs",
    "CGState", "cg_direction", "ml_cycle", "simulate_intensity", "UPDATE_OBJECT",
    "UPDATE_PROBE", "UPDATE_BACKGROUND", "DEFAULT_EPS", "DEFAULT_INERTIA",
    "model_intensity", "projection_scale", "background_update",
    "object_gradient", "position_shifts", "ml_position_shifts", "update_positions",
    "windows_from_positions", "views_adjoint",
    "fresnel_pair", "near_field_transfer", "propagate_near_field", "to_detector", "from_detector",
]

UPDATE_OBJECT = 1
UPDATE_PROBE = 2
UPDATE_BACKGROUND = 4        # AP only: refine the incoherent background
DEFAULT_EPS = 1e-20          # floor on the calculated intensity
DEFAULT_INERTIA = 1e-2       # delta in alpha = delta * max(denominator)


# --------------------------------------------------------------------------
# Propagation (appendix table of ptychography operators: FT / IFT)
# --------------------------------------------------------------------------

def fft2(x: np.ndarray) -> np.ndarray:
    """Unitary forward 2D DFT over the last two axes, sign -1, q=0 at [0,0].

    The paper does not fix the normalisation; the unitary one keeps the
    observed intensities in photons and makes the propagator its own
    adjoint's inverse.
    """
    return np.fft.fft2(np.asarray(x, dtype=np.complex128), norm="ortho")


def ifft2(x: np.ndarray) -> np.ndarray:
    """Unitary inverse 2D DFT over the last two axes."""
    return np.fft.ifft2(np.asarray(x, dtype=np.complex128), norm="ortho")


def fresnel_pair(nf) -> tuple:
    """(f_y, f_x) from a scalar (square pixels) or a pair."""
    f = np.broadcast_to(np.asarray(nf, dtype=np.float64), (2,))
    return float(f[0]), float(f[1])


def near_field_transfer(n: int, nf) -> np.ndarray:
    """Fresnel transfer function on the N x N DFT grid (FFT order):
    Q[u, v] = exp(-i (f_y u'^2 + f_x v'^2)), u' = u for u < N/2 else u - N.

    Operator PropagateNearField.  The paper names the operator but not its
    formula; the reading taken is the paraxial (Fresnel) transfer function
    exp(-i pi lambda z |q|^2) of a field with exp(+ikz) dependence, the
    constant exp(ikz) dropped.  With q = u'/(N dx) the phase is f u'^2 with the
    dimensionless f = pi lambda z / (N dx)^2 per axis; a magnified (cone-beam)
    geometry enters through its effective distance.
    """
    fy, fx = fresnel_pair(nf)
    u = np.fft.fftfreq(n) * n
    return np.exp(-1j * (fy * u[:, None] ** 2 + fx * u[None, :] ** 2))


def propagate_near_field(x: np.ndarray, nf, direction: int = 1) -> np.ndarray:
    """Near-field propagation over the last two axes: F^-1 Q F (direction +1,
    sample to detector) or F^-1 conj(Q) F (-1, back to the sample).  Unitary,
    and the two directions are each other's inverse."""
    q = near_field_transfer(np.asarray(x).shape[-1], nf)
    if direction < 0:
        q = np.conj(q)
    return ifft2(fft2(x) * q)


def to_detector(x: np.ndarray, nf=None) -> np.ndarray:
    """Sample plane -> detector plane: the far-field FT (nf None), else
    near-field propagation with Fresnel parameter(s) nf.  Both are unitary,
    so every formula below holds with either in place of F."""
    return fft2(x) if nf is None else propagate_near_field(x, nf, +1)


def from_detector(x: np.ndarray, nf=None) -> np.ndarray:
    """Inverse (= adjoint) of `to_detector`."""
    return ifft2(x) if nf is None else propagate_near_field(x, nf, -1)


# --------------------------------------------------------------------------
# Scan positions and views (Section 4, PtychoData; operator ObjProbe2Psi)
# --------------------------------------------------------------------------

def offsets_from_positions(pos_yx: np.ndarray, n: int, obj_shape) -> np.ndarray:
    """Integer top-left window corner of each scan position.

    Positions are in pixels relative to the object centre (Ny/2, Nx/2).  The
    window of frame j starts at floor(centre + p_j + 1/2) - N/2 along each
    axis (round half up, never half to even).  A window that does not fit in
    the object is an error, never clamped.
    """
    pos = np.asarray(pos_yx, dtype=np.float64)
    ny, nx = obj_shape
    centre = np.array([ny / 2.0, nx / 2.0])
    o = np.floor(centre[None, :] + pos + 0.5).astype(np.int64) - n // 2
    if o.size and (o.min() < 0 or (o[:, 0] > ny - n).any() or (o[:, 1] > nx - n).any()):
        raise ValueError("scan position window outside the object")
    return o.astype(np.int32)


def windows_from_positions(pos_yx: np.ndarray, n: int, obj_shape):
    """Sub-pixel windows: the real top-left corner t = centre + p - N/2 of each
    frame split into its integer part o = floor(t) and fraction f = t - o in
    [0, 1), per axis.  Reading: refined positions are real numbers (the
    position optimisation of Section 4 moves them by fractions of a pixel), and
    a window at a fractional corner views the object by bilinear
    interpolation (`views`).  A corner outside [0, Ny - N] x [0, Nx - N] is an
    error.  Returns (offsets int32 [J][2], frac float64 [J][2])."""
    pos = np.asarray(pos_yx, dtype=np.float64)
    ny, nx = obj_shape
    t = np.array([ny / 2.0, nx / 2.0])[None, :] + pos - n / 2.0
    if t.size and (t.min() < 0 or (t[:, 0] > ny - n).any() or (t[:, 1] > nx - n).any()):
        raise ValueError("scan position window outside the object")
    o = np.floor(t)
    return o.astype(np.int32), t - o


def views(obj: np.ndarray, offsets: np.ndarray, n: int, frac=None) -> np.ndarray:
    """Object patches under each frame window: [J][N][N].

    With frac (sub-pixel windows, `windows_from_positions`) the patch is the
    bilinear interpolation of the object at (o + f + y, o + f + x):
      V[y, x] = sum over a, b in {0, 1} of w_a(f_y) w_b(f_x) O[o_y + y + a, o_x + x + b]
    with w_0(f) = 1 - f, w_1(f) = f.  A neighbour beyond the object's last row
    or column only ever has weight 0 (the corner is at most Ny - N) and is
    read at the border instead."""
    obj = np.asarray(obj)
    if frac is None:
        return np.stack([obj[oy:oy + n, ox:ox + n] for oy, ox in offsets])
    ny, nx = obj.shape
    out = []
    for (oy, ox), (fy, fx) in zip(offsets, np.asarray(frac, dtype=np.float64)):
        rows = np.minimum(np.arange(oy, oy + n + 1), ny - 1)
        cols = np.minimum(np.arange(ox, ox + n + 1), nx - 1)
        w = obj[np.ix_(rows, cols)]
        out.append((1 - fy) * (1 - fx) * w[:n, :n] + (1 - fy) * fx * w[:n, 1:] +
                   fy * (1 - fx) * w[1:, :n] + fy * fx * w[1:, 1:])
    return np.stack(out)


def views_adjoint(planes: np.ndarray, offsets: np.ndarray, obj_shape, frac=None) -> np.ndarray:
    """Adjoint of `views`: sum over frames of each plane [N][N] put back on
    the object grid, i.e. S_j^T applied to plane j and summed.  Integer
    windows add plane j to the object window; sub-pixel windows spread
    plane[y, x] over the four object pixels its bilinear view reads, with the
    same weights (terms that would fall beyond the object have weight 0)."""
    planes = np.asarray(planes)
    n = planes.shape[-1]
    out = np.zeros(obj_shape, dtype=planes.dtype)
    if frac is None:
        for (oy, ox), pl in zip(offsets, planes):
            out[oy:oy + n, ox:ox + n] += pl
        return out
    ny, nx = obj_shape
    for (oy, ox), (fy, fx), pl in zip(offsets, np.asarray(frac, dtype=np.float64), planes):
        for a, wa in ((0, 1 - fy), (1, fy)):
            for b, wb in ((0, 1 - fx), (1, fx)):
                if wa * wb == 0.0:
                    continue
                out[oy + a:oy + a + n, ox + b:ox + b + n] += (wa * wb) * pl
    return out


def exit_waves(obj: np.ndarray, probe: np.ndarray, offsets: np.ndarray, frac=None) -> np.ndarray:
    """Exit waves Psi_jk(r) = O(r + o_j) P_k(r) (ptychography operator table,
    ObjProbe2Psi: the object times the probe shifted to position j), with
    sub-pixel windows when frac is given."""
    probe = np.asarray(probe, dtype=np.complex128)
    v = views(np.asarray(obj, dtype=np.complex128), offsets, probe.shape[-1], frac)
    return v[:, None, :, :] * probe[None, :, :, :]


def psi_init(obj, probe, offsets, frac=None) -> np.ndarray:
    """DM starting exit waves: the current views (Psi^0 = Phi^0)."""
    return exit_waves(obj, probe, offsets, frac)


# --------------------------------------------------------------------------
# Modulus projection (operator ApplyAmplitude / PropagateApplyAmplitude)
# --------------------------------------------------------------------------

def calc_intensity(psi_hat: np.ndarray) -> np.ndarray:
    """Calculated intensity: incoherent sum over probe modes, [J][N][N]."""
    return (np.abs(psi_hat) ** 2).sum(axis=1)


def model_intensity(psi_hat: np.ndarray, bg=None) -> np.ndarray:
    """Model intensity: the modes' sum plus the incoherent background bg
    [N][N] (shared by all frames, in the detector layout of iobs), which the Ptycho object of
    Section 4 carries beside object and probe; bg None means zero."""
    inten = calc_intensity(psi_hat)
    return inten if bg is None else inten + np.asarray(bg, dtype=np.float64)[None]


def projection_scale(psi_hat, iobs, mask, eps=DEFAULT_EPS, bg=None) -> np.ndarray:
    """s = sqrt(Iobs / I) per frame and pixel, I the model intensity floored
    at eps; 1 at bad pixels."""
    inten = model_intensity(psi_hat, bg)
    scale = np.sqrt(np.asarray(iobs, dtype=np.float64) / np.maximum(inten, eps))
    if mask is not None:
        scale = np.where(np.asarray(mask)[None, :, :] != 0, 1.0, scale)
    return scale


def project_modulus(psi_hat: np.ndarray, iobs: np.ndarray,
                    mask: Optional[np.ndarray], eps: float = DEFAULT_EPS, bg=None) -> np.ndarray:
    """Replace the Fourier modulus by the observed amplitude.

    With several incoherent probe modes all modes of a pixel share one scale
    sqrt(Iobs / I), I = sum_k |Psi_k|^2 (+ background) floored at eps, so
    that the projected model (modes and background, the background taken as
    one more incoherent mode) matches the observed intensity and the modes
    keep their phases.  Bad (masked) pixels are left unchanged.
    """
    return psi_hat * projection_scale(psi_hat, iobs, mask, eps, bg)[:, None, :, :]


def fourier_project(psi: np.ndarray, iobs, mask, eps: float = DEFAULT_EPS, bg=None, nf=None) -> np.ndarray:
    """PropagateApplyAmplitude on every frame and mode: IFT * ApplyAmplitude *
    FT in the far field, or the same with near-field propagation both ways
    (nf given), the amplitude then replaced in the detector plane."""
    return from_detector(project_modulus(to_detector(psi, nf), iobs, mask, eps, bg), nf)


def background_update(bg, scale) -> np.ndarray:
    """Incoherent background refinement of AP (Section 4, after Marchesini et
    al. 2013).  Reading: the background is the one incoherent mode that all
    frames share, so its projected intensity at frame j is bg * s_j^2 and the
    new background is the mean of that over the frames:
      bg' = bg * (1/J) sum_j s_j^2
    (s = 1 at bad pixels, which keep their value)."""
    return np.asarray(bg, dtype=np.float64) * (np.asarray(scale) ** 2).mean(axis=0)


# --------------------------------------------------------------------------
# Object / probe update (operator Psi2ObjProbe; inertia, Section 4)
# --------------------------------------------------------------------------

def overlap_sums(psi, obj, probe, offsets, frac=None):
    """Numerators and denominators of the overlap (least-squares) update.

    numO(r) = sum_jk conj(P_k(r - o_j)) Psi_jk(r - o_j)
    denO(r) = sum_jk |P_k(r - o_j)|^2
    numP_k(r) = sum_j conj(O(r + o_j)) Psi_jk(r)
    denP(r) = sum_j |O(r + o_j)|^2
    numO and denO use the given probe, numP and denP the given object.  With
    sub-pixel windows (frac) the object terms go back through the adjoint of
    the bilinear view, numO = sum_j S_j^T (sum_k conj(P_k) Psi_jk) and
    denO = sum_j S_j^T (sum_k |P_k|^2): the row sums of the normal matrix
    sum_j S_j^T diag(sum_k |P_k|^2) S_j, which is not diagonal once windows
    interpolate (reading: the update keeps a diagonal denominator, exact for
    integer windows); numP and denP use the interpolated views.
    """
    psi = np.asarray(psi, dtype=np.complex128)
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    n = probe.shape[-1]
    p_conj = np.conj(probe)
    p_int = (np.abs(probe) ** 2).sum(axis=0)
    q = np.stack([(p_conj * psi[j]).sum(axis=0) for j in range(len(offsets))])
    num_o = views_adjoint(q, offsets, obj.shape, frac)
    den_o = views_adjoint(np.broadcast_to(p_int, (len(offsets), n, n)), offsets, obj.shape, frac)
    v = views(obj, offsets, n, frac)
    num_p = np.zeros(probe.shape, dtype=np.complex128)
    den_p = np.zeros(probe.shape[1:], dtype=np.float64)
    for j in range(len(offsets)):
        num_p += np.conj(v[j])[None] * psi[j]
        den_p += np.abs(v[j]) ** 2
    return num_o, den_o, num_p, den_p


def overlap_denominators(obj, probe, offsets, frac=None):
    """denO and denP alone (they do not depend on the exit waves)."""
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    n = probe.shape[-1]
    p_int = (np.abs(probe) ** 2).sum(axis=0)
    den_o = views_adjoint(np.broadcast_to(p_int, (len(offsets), n, n)), offsets, obj.shape, frac)
    den_p = np.zeros(probe.shape[1:], dtype=np.float64)
    for v in views(obj, offsets, n, frac):
        den_p += np.abs(v) ** 2
    return den_o, den_p


def overlap_update(obj, probe, psi, offsets, update=UPDATE_OBJECT | UPDATE_PROBE,
                   inertia_obj=DEFAULT_INERTIA, inertia_probe=DEFAULT_INERTIA, frac=None):
    """New object and probe from the exit waves (Psi2ObjProbe).

    The object is updated first, from the current probe; the probe is then
    updated from the *new* object (one Gauss-Seidel sweep; the paper does not
    say).  Updating both from the same old pair instead lets each factor absorb
    the same scale, so their product overshoots and the DM iteration diverges
    (tests/test_oracle_pins.py shows it).  The inertia of Section 4 enters as
    a regularising weight alpha = delta * max(den) that pulls each pixel
    towards its previous value:  O <- (numO + a_O O) / (denO + a_O).  A pixel
    whose denominator is exactly zero (never illuminated, no inertia) keeps
    its value.
    """
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    new_obj, new_probe = obj.copy(), probe.copy()
    if update & UPDATE_OBJECT:
        num_o, den_o, _, _ = overlap_sums(psi, obj, probe, offsets, frac)
        a = inertia_obj * den_o.max()
        d = den_o + a
        new_obj = np.where(d > 0, (num_o + a * obj) / np.where(d > 0, d, 1.0), obj)
    if update & UPDATE_PROBE:
        _, _, num_p, den_p = overlap_sums(psi, new_obj, probe, offsets, frac)
        a = inertia_probe * den_p.max()
        d = (den_p + a)[None]
        new_probe = np.where(d > 0, (num_p + a * probe) / np.where(d > 0, d, 1.0), probe)
    return new_obj, new_probe


# --------------------------------------------------------------------------
# Projection algorithms (operators AP and DM; Section 4 algorithm list)
# --------------------------------------------------------------------------

def ap_cycle(obj, probe, offsets, iobs, mask, update=UPDATE_OBJECT | UPDATE_PROBE,
             inertia_obj=DEFAULT_INERTIA, inertia_probe=DEFAULT_INERTIA,
             eps=DEFAULT_EPS, bg=None, nf=None, frac=None):
    """One alternating-projections cycle: views, Fourier projection of every
    frame, then one object/probe update from all projected exit waves.
    Returns (obj, probe); with a background bg, (obj, probe, bg), the
    background refined by `background_update` when UPDATE_BACKGROUND is set.
    nf: near-field Fresnel parameter(s) (`near_field_transfer`), None = far
    field."""
    if (update & UPDATE_BACKGROUND) and bg is None:
        raise ValueError("a background update needs a background")
    phi = exit_waves(obj, probe, offsets, frac)
    phi_hat = to_detector(phi, nf)
    scale = projection_scale(phi_hat, iobs, mask, eps, bg)
    psi = from_detector(phi_hat * scale[:, None, :, :], nf)
    o, p = overlap_update(obj, probe, psi, offsets, update & (UPDATE_OBJECT | UPDATE_PROBE),
                          inertia_obj, inertia_probe, frac)
    if bg is None:
        return o, p
    b = background_update(bg, scale) if update & UPDATE_BACKGROUND else np.asarray(bg, dtype=np.float64)
    return o, p, b


def dm_cycle(obj, probe, psi, offsets, iobs, mask, update=UPDATE_OBJECT | UPDATE_PROBE,
             inertia_obj=DEFAULT_INERTIA, inertia_probe=DEFAULT_INERTIA,
             eps=DEFAULT_EPS, bg=None, nf=None, frac=None):
    """One difference-map cycle (beta = 1) on persistent exit waves.

    Phi = views of the current object and probe (the overlap projection of
    the previous cycle's Psi); Psi <- Psi + P_F(2 Phi - Psi) - Phi; then the
    object and probe are updated from the new Psi.  Returns (obj, probe, psi).
    """
    phi = exit_waves(obj, probe, offsets, frac)
    psi = np.asarray(psi, dtype=np.complex128)
    psi_new = psi + fourier_project(2.0 * phi - psi, iobs, mask, eps, bg, nf) - phi
    o, p = overlap_update(obj, probe, psi_new, offsets, update, inertia_obj, inertia_probe, frac)
    return o, p, psi_new


# --------------------------------------------------------------------------
# Poisson log-likelihood (operator LLK; Section 4, noise models)
# --------------------------------------------------------------------------

def llk_terms(icalc, iobs, eps=DEFAULT_EPS):
    """Per-pixel Poisson negative log-likelihood relative to a perfect fit:
    I - Iobs + Iobs ln(Iobs / I), with 0 ln 0 = 0 and I floored at eps."""
    i = np.maximum(np.asarray(icalc, dtype=np.float64), eps)
    o = np.asarray(iobs, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(o > 0, o * np.log(o / i), 0.0)
    return i - o + t


LLK_MODELS = ("poisson", "gaussian", "euclidean")


def llk_model_terms(icalc, iobs, model, eps=DEFAULT_EPS):
    """Per-pixel negative log-likelihood, up to a constant, of the three noise
    models the paper reports the likelihood for (Section 4, after Thibault &
    Guizar-Sicairos 2012):
      poisson   : I - Iobs + Iobs ln(Iobs / I)        (deviance / 2)
      gaussian  : (I - Iobs)^2 / (2 (Iobs + 1))       (variance Iobs + 1)
      euclidean : 2 (sqrt(I) - sqrt(Iobs))^2          (amplitude variance 1/4)
    Reading: each is the negative log of its density with the constant that
    makes it zero at a perfect fit, so all three agree to second order near
    the fit (about Iobs d^2 / 2 for I = Iobs (1 + d)).  I is floored at eps."""
    i = np.maximum(np.asarray(icalc, dtype=np.float64), eps)
    o = np.asarray(iobs, dtype=np.float64)
    if model == "poisson":
        return llk_terms(i, o, eps)
    if model == "gaussian":
        return (i - o) ** 2 / (2.0 * (o + 1.0))
    if model == "euclidean":
        return 2.0 * (np.sqrt(i) - np.sqrt(np.maximum(o, 0.0))) ** 2
    raise ValueError(f"unknown noise model {model!r}")


def llk(obj, probe, offsets, iobs, mask, eps=DEFAULT_EPS, model="poisson", bg=None, nf=None, frac=None):
    """(sum over unmasked pixels of all frames, number of those pixels) of
    the chosen noise model's terms."""
    inten = model_intensity(to_detector(exit_waves(obj, probe, offsets, frac), nf), bg)
    terms = llk_model_terms(inten, iobs, model, eps)
    if mask is not None:
        good = np.broadcast_to(np.asarray(mask)[None] == 0, terms.shape)
    else:
        good = np.ones(terms.shape, dtype=bool)
    return float(terms[good].sum()), int(good.sum())


def ml_grad(obj, probe, offsets, iobs, mask, eps=DEFAULT_EPS, bg=None, nf=None, frac=None):
    """Gradient of the Poisson LLK w.r.t. object and probe.

    Convention: g = dL/dRe(z) + i dL/dIm(z) (= 2 dL/dz*).  With
    Psi^_jk = F(P_k O_j), I_j = sum_k |Psi^_jk|^2 (+ bg) and l'(I) = 1 - Iobs/I
    (0 at bad pixels), the chain rule through the unitary F gives
      psi_jk = F^-1(l'(I_j) Psi^_jk)
      g_O = 2 sum_jk S_j^T (conj(P_k) psi_jk)
      g_P_k = 2 sum_j conj(O_j) psi_jk
    In the near field (nf given) F is the unitary propagation and F^-1 its
    adjoint.  With sub-pixel windows (frac) S_j is the bilinear view and
    S_j^T its adjoint (`views_adjoint`), so the gradient stays exact.
    Returns (g_obj, g_probe, llk_sum).
    """
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    n = probe.shape[-1]
    phi_hat = to_detector(exit_waves(obj, probe, offsets, frac), nf)
    inten = np.maximum(model_intensity(phi_hat, bg), eps)
    io = np.asarray(iobs, dtype=np.float64)
    dl = 1.0 - io / inten
    terms = llk_terms(inten, io, eps)
    if mask is not None:
        bad = np.asarray(mask)[None] != 0
        dl = np.where(bad, 0.0, dl)
        terms = np.where(bad, 0.0, terms)
    psi = from_detector(dl[:, None] * phi_hat, nf)
    p_conj = np.conj(probe)
    q = np.stack([(p_conj * psi[j]).sum(axis=0) for j in range(len(offsets))])
    g_o = 2.0 * views_adjoint(q, offsets, obj.shape, frac)
    g_p = np.zeros(probe.shape, dtype=np.complex128)
    for j, v in enumerate(views(obj, offsets, n, frac)):
        g_p += 2.0 * np.conj(v)[None] * psi[j]
    return g_o, g_p, float(terms.sum())


def linesearch_coefs(obj, probe, dobj, dprobe, offsets, iobs, mask, eps=DEFAULT_EPS, bg=None, nf=None,
                     frac=None):
    """First and second derivative of L(gamma) = LLK(O + g dO, P + g dP) at 0.

    The exit wave along the line is A + gamma B + gamma^2 C with
    A = F(P O_j), B = F(P dO_j + dP O_j), C = F(dP dO_j), so
      I(gamma) = I0 + gamma I1 + gamma^2 I2 + O(gamma^3)
      I1 = 2 Re sum_k conj(A_k) B_k,   I2 = sum_k |B_k|^2 + 2 Re sum_k conj(A_k) C_k
      L'(0) = sum l'(I0) I1,  L''(0) = sum [l''(I0) I1^2 + 2 l'(I0) I2]
    with l' = 1 - Iobs/I0, l'' = Iobs/I0^2, both 0 at bad pixels (the
    quadratic line search of the Poisson ML conjugate gradient the paper
    cites, Thibault & Guizar-Sicairos 2012).
    """
    a = to_detector(exit_waves(obj, probe, offsets, frac), nf)
    b = to_detector(exit_waves(obj, dprobe, offsets, frac) + exit_waves(dobj, probe, offsets, frac), nf)
    c = to_detector(exit_waves(dobj, dprobe, offsets, frac), nf)
    i0 = np.maximum(model_intensity(a, bg), eps)
    i1 = 2.0 * (np.conj(a) * b).real.sum(axis=1)
    i2 = (np.abs(b) ** 2).sum(axis=1) + 2.0 * (np.conj(a) * c).real.sum(axis=1)
    io = np.asarray(iobs, dtype=np.float64)
    d1 = 1.0 - io / i0
    d2 = io / (i0 * i0)
    if mask is not None:
        bad = np.asarray(mask)[None] != 0
        d1 = np.where(bad, 0.0, d1)
        d2 = np.where(bad, 0.0, d2)
    return float((d1 * i1).sum()), float((d2 * i1 * i1 + 2.0 * d1 * i2).sum())


# --------------------------------------------------------------------------
# Conjugate-gradient ML cycle (operator ML)
# --------------------------------------------------------------------------

def _dot(a, b) -> float:
    """Real inner product Re sum conj(a) b."""
    return float(np.vdot(a, b).real)


@dataclass
class CGState:
    """Search direction and previous gradient carried between ML cycles."""
    d_obj: Optional[np.ndarray] = None
    d_probe: Optional[np.ndarray] = None
    g_obj: Optional[np.ndarray] = None
    g_probe: Optional[np.ndarray] = None
    zg: float = 0.0
    history: list = field(default_factory=list)


def cg_direction(state: CGState, g_o, g_p, s: float):
    """Search direction of one preconditioned Polak-Ribiere (PR+) step.

    Operator ML's conjugate gradient (Section 4, after Thibault and
    Guizar-Sicairos 2012).  The preconditioner scales the probe block by s:
    z = (g_O, s g_P).  With the previous gradient and direction in `state`,
      beta = max(0, <z_n, g_n - g_{n-1}> / <z_{n-1}, g_{n-1}>)
    (Polak-Ribiere, restarted at 0 whenever it is negative), beta = 0 when no
    previous direction exists, and d = -z + beta d_prev, where
    <a, b> = Re sum conj(a) b over the object and probe blocks.  Updates
    `state` (direction, gradient, <z, g>) and returns (d_O, d_P, beta).
    """
    zg = _dot(g_o, g_o) + s * _dot(g_p, g_p)
    if state.d_obj is None or state.zg <= 0.0:
        beta = 0.0
        d_o = -g_o
        d_p = -s * g_p
    else:
        num = _dot(g_o, g_o - state.g_obj) + s * _dot(g_p, g_p - state.g_probe)
        beta = max(0.0, num / state.zg)
        d_o = -g_o + beta * state.d_obj
        d_p = -s * g_p + beta * state.d_probe
    state.d_obj, state.d_probe = d_o, d_p
    state.g_obj, state.g_probe = g_o, g_p
    state.zg = zg
    return d_o, d_p, beta


def ml_cycle(obj, probe, state: CGState, offsets, iobs, mask,
             update=UPDATE_OBJECT, eps=DEFAULT_EPS, bg=None, nf=None, frac=None):
    """One Polak-Ribiere (PR+) conjugate-gradient step on the Poisson LLK.

    The probe block of the gradient is scaled by s = max(denO) / max(denP)
    (a diagonal preconditioner that balances object and probe steps) and the
    direction comes from `cg_direction`; the step gamma = -L'(0)/L''(0)
    from `linesearch_coefs` (0 when L''(0) <= 0).  Blocks not being updated
    have zero gradient.  Returns (obj, probe) and updates `state` in place;
    `state.history` receives the LLK at the start of the cycle.
    """
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    g_o, g_p, lsum = ml_grad(obj, probe, offsets, iobs, mask, eps, bg, nf, frac)
    if not update & UPDATE_OBJECT:
        g_o = np.zeros_like(g_o)
    if not update & UPDATE_PROBE:
        g_p = np.zeros_like(g_p)
    den_o, den_p = overlap_denominators(obj, probe, offsets, frac)
    s = den_o.max() / den_p.max() if den_p.max() > 0 else 1.0
    d_o, d_p, _ = cg_direction(state, g_o, g_p, s)
    l1, l2 = linesearch_coefs(obj, probe, d_o, d_p, offsets, iobs, mask, eps, bg, nf, frac)
    gamma = -l1 / l2 if (l2 > 0.0 and math.isfinite(l1) and math.isfinite(l2)) else 0.0
    state.history.append(lsum)
    return obj + gamma * d_o, probe + gamma * d_p


# --------------------------------------------------------------------------
# Position refinement (operator Psi2PosShift; Section 4, after Odstrcil et
# al. 2018)
# --------------------------------------------------------------------------

def object_gradient(obj):
    """(dO/dy, dO/dx) on the object grid: centred differences inside,
    one-sided differences on the object's border (numpy.gradient)."""
    o = np.asarray(obj, dtype=np.complex128)
    return np.gradient(o, axis=0), np.gradient(o, axis=1)


def position_shifts(obj, probe, psi, offsets, frac=None):
    """Shift of every frame's illumination position from its exit waves.

    A frame whose true position is r_j + d has exit waves
    P_k O(r + r_j + d) ~ P_k O_j + d . P_k grad O_j, so the difference
    chi_jk = Psi_jk - P_k O_j between the given exit waves and the current
    views is fitted by least squares in the two components of d together
    (reading: the gradient-based shift of Odstrcil et al. 2018 solved as one
    2x2 system, since the y and x gradients of a small window correlate):
      [S_yy S_yx] [d_y]   [sum Re(conj(G_y) chi)]
      [S_xy S_xx] [d_x] = [sum Re(conj(G_x) chi)],  S_ab = sum Re(conj(G_a) G_b)
    with G_a = P_k dO/da over frame j's window and the sums over modes and
    pixels (d = 0 when the system is singular).  With sub-pixel windows
    (frac) the view and the gradient are both interpolated bilinearly.  Also
    returns the frame's gradient energy e_j = S_yy + S_xx, by which frames
    with too little object contrast are left in place.
    Returns (shifts [J][2] as (dy, dx) in pixels, e [J])."""
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    psi = np.asarray(psi, dtype=np.complex128)
    gy, gx = object_gradient(obj)
    n = probe.shape[-1]
    vo, vy, vx = (views(a, offsets, n, frac) for a in (obj, gy, gx))
    shifts = np.zeros((len(offsets), 2))
    energy = np.zeros(len(offsets))
    for j in range(len(offsets)):
        chi = psi[j] - probe * vo[j][None]
        g = [probe * vy[j][None], probe * vx[j][None]]
        a = np.array([[float((np.conj(g[r]) * g[c]).real.sum()) for c in range(2)] for r in range(2)])
        b = np.array([float((np.conj(g[r]) * chi).real.sum()) for r in range(2)])
        det = a[0, 0] * a[1, 1] - a[0, 1] * a[1, 0]
        if det > 1e-12 * a[0, 0] * a[1, 1] and det > 0:
            shifts[j] = np.linalg.solve(a, b)
        energy[j] = a[0, 0] + a[1, 1]
    return shifts, energy


def ml_position_shifts(obj, probe, offsets, iobs, mask, eps=DEFAULT_EPS, bg=None, nf=None, frac=None):
    """Position shifts during ML (Section 4: position optimisation during AP
    and ML).  Reading: the exit-wave change that ML proposes is minus half the
    back-propagated gradient wave, chi = -1/2 F^-1(l'(I) F(Phi)) with
    l' = 1 - Iobs/I (0 at bad pixels), which near the fit equals the AP
    correction F^-1((s - 1) F(Phi)) to first order (1 - s^2 ~ -2 (s - 1) for
    s = sqrt(Iobs/I)); the shifts are `position_shifts` of Phi + chi at the
    current object, probe and windows."""
    obj = np.asarray(obj, dtype=np.complex128)
    probe = np.asarray(probe, dtype=np.complex128)
    phi = exit_waves(obj, probe, offsets, frac)
    phi_hat = to_detector(phi, nf)
    inten = np.maximum(model_intensity(phi_hat, bg), eps)
    dl = 1.0 - np.asarray(iobs, dtype=np.float64) / inten
    if mask is not None:
        dl = np.where(np.asarray(mask)[None] != 0, 0.0, dl)
    chi = -0.5 * from_detector(dl[:, None] * phi_hat, nf)
    return position_shifts(obj, probe, phi + chi, offsets, frac)


def update_positions(pos, pos0, shifts, energy, mult=1.0, max_shift=2.0, min_grad=0.1):
    """New positions pos + mult * shift, where frames whose gradient energy
    is below min_grad times the median energy are not moved (the filter the
    paper adds against low object contrast), and the total move from the
    starting positions pos0 is clipped to +-max_shift pixels per axis."""
    pos = np.asarray(pos, dtype=np.float64)
    pos0 = np.asarray(pos0, dtype=np.float64)
    keep = np.asarray(energy) >= min_grad * np.median(energy)
    new = pos + mult * np.where(keep[:, None], np.asarray(shifts), 0.0)
    return pos0 + np.clip(new - pos0, -max_shift, max_shift)


# --------------------------------------------------------------------------
# Forward model for simulation (Section 4, simulation functions)
# --------------------------------------------------------------------------

def simulate_intensity(obj, probe, offsets, chunk: int = 64, bg=None, nf=None, frac=None) -> np.ndarray:
    """Noise-free intensities sum_k |F(P_k O_j)|^2 (+ bg), float64 [J][N][N]:
    far field (FFT order), or near field with Fresnel parameter(s) nf
    (detector pixels in natural order)."""
    out = []
    for s in range(0, len(offsets), chunk):
        fr = None if frac is None else np.asarray(frac)[s:s + chunk]
        out.append(model_intensity(to_detector(exit_waves(obj, probe, offsets[s:s + chunk], fr), nf), bg))
    return np.concatenate(out, axis=0)

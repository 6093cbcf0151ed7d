"""Torch-facing wrapper of a ptychography plan (marshalling only)."""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FLAG_BACKGROUND, FLAG_NEAR_FIELD, FLAG_POSITIONS, Desc, check, lib


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _need(t: torch.Tensor, name: str, dtype, shape, device) -> None:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def offsets_from_positions(pos_yx, n: int, obj_shape) -> np.ndarray:
    """Scan positions (pixels from the object centre) -> int32 window corners
    (host computation inside the library)."""
    pos = np.ascontiguousarray(pos_yx, dtype=np.float64)
    j = pos.shape[0]
    out = np.empty((j, 2), dtype=np.int32)
    check(lib().ptycho_offsets_from_positions(pos.ctypes.data, j, int(n), int(obj_shape[0]),
                                              int(obj_shape[1]), out.ctypes.data))
    return out


def windows_from_positions(pos_yx, n: int, obj_shape):
    """Scan positions (pixels from the object centre) -> (int32 window
    corners [J][2], float64 fractions [J][2]) of sub-pixel windows (host
    computation inside the library)."""
    pos = np.ascontiguousarray(pos_yx, dtype=np.float64)
    j = pos.shape[0]
    offs = np.empty((j, 2), dtype=np.int32)
    frac = np.empty((j, 2), dtype=np.float64)
    check(lib().ptycho_windows_from_positions(pos.ctypes.data, j, int(n), int(obj_shape[0]), int(obj_shape[1]),
                                              offs.ctypes.data, frac.ctypes.data))
    return offs, frac


def update_positions(pos: torch.Tensor, pos0: torch.Tensor, shifts: torch.Tensor, mult: float = 1.0,
                     max_shift: float = 2.0, min_grad: float = 0.1, out: Optional[torch.Tensor] = None):
    """New scan positions (float64 [J][2] device tensor, pixels) from the
    shifts of `Plan.position_shifts` (float64 [J][3]), computed by the
    library on the current stream: the low-contrast filter, the step and
    the bound on the total move from pos0 (see ptycho_update_positions)."""
    j = pos.shape[0]
    for name, t, shape in (("pos", pos, (j, 2)), ("pos0", pos0, (j, 2)), ("shifts", shifts, (j, 3))):
        _need(t, name, torch.float64, shape, pos.device)
    out = torch.empty_like(pos) if out is None else out
    _need(out, "out", torch.float64, (j, 2), pos.device)
    check(lib().ptycho_update_positions(j, _ptr(pos), _ptr(pos0), _ptr(shifts), float(mult), float(max_shift),
                                        float(min_grad), _ptr(out),
                                        torch.cuda.current_stream(pos.device).cuda_stream))
    return out


def refine_positions(plan: "Plan", obj, probe, psi, pos, pos0, mult: float = 1.0, max_shift: float = 2.0,
                     min_grad: float = 0.1):
    """One position-refinement step after a cycle that left exit waves in psi:
    the shifts and the position update in the library, then a plan rebuilt
    on the new offsets when any frame moved to another pixel.
    Returns (plan, new positions, new offsets)."""
    sh = plan.position_shifts(obj, probe, psi)
    pos_d = torch.as_tensor(np.ascontiguousarray(pos, dtype=np.float64)).to(plan.device)
    pos0_d = torch.as_tensor(np.ascontiguousarray(pos0, dtype=np.float64)).to(plan.device)
    new = update_positions(pos_d, pos0_d, sh, mult, max_shift, min_grad).cpu().numpy()
    offs = offsets_from_positions(new, plan.n, plan.obj_shape)
    if not np.array_equal(offs, plan.offsets):
        plan = plan.rebuild(offs)
    return plan, new, offs


def fft2(x: torch.Tensor, inverse: bool = False) -> torch.Tensor:
    """Unitary batched 2D FFT over the last two axes (in place on a copy)."""
    if x.dtype != torch.complex64 or not x.is_cuda:
        raise TypeError("fft2 takes a complex64 CUDA tensor")
    y = x.contiguous().clone()
    n = y.shape[-1]
    if y.shape[-2] != n:
        raise ValueError("frames must be square")
    count = y.numel() // (n * n)
    check(lib().ptycho_fft2(n, count, _ptr(y), 1 if inverse else -1,
                            torch.cuda.current_stream(y.device).cuda_stream))
    return y


class Plan:
    """One scan: positions, observed intensities and mask on one device.

    Tensors: iobs float32 [J][N][N] (FFT order; near field: natural pixel
    order), mask uint8 [N][N] or None, obj complex64 [Ny][Nx], probe
    complex64 [K][N][N], psi complex64 [J][K][N][N].  Work is enqueued on the
    current torch stream at call time.  near_field: Fresnel parameter f, or
    (f_y, f_x), selecting the near-field geometry (f = pi lambda z / (N dx)^2);
    None = far field.
    """

    def __init__(self, offsets, iobs: torch.Tensor, mask: Optional[torch.Tensor], n_modes: int,
                 obj_shape, stack: int = 0, obj_inertia: float = 1e-2, probe_inertia: float = 1e-2,
                 icalc_floor: float = 1e-20, workspace: Optional[torch.Tensor] = None,
                 background_update: bool = False, near_field=None, max_shift: Optional[float] = None):
        offs = np.ascontiguousarray(offsets, dtype=np.int32)
        if offs.ndim != 2 or offs.shape[1] != 2:
            raise ValueError("offsets must be [J][2]")
        j = offs.shape[0]
        if iobs.ndim != 3:
            raise ValueError("iobs must be [J][N][N]")
        n = int(iobs.shape[-1])
        self.device = iobs.device
        _need(iobs, "iobs", torch.float32, (j, n, n), self.device)
        if mask is not None:
            _need(mask, "mask", torch.uint8, (n, n), self.device)
        self.n, self.k, self.j = n, int(n_modes), j
        self.obj_shape = (int(obj_shape[0]), int(obj_shape[1]))
        self.desc = Desc(n, self.k, j, self.obj_shape[0], self.obj_shape[1], int(stack),
                         float(obj_inertia), float(probe_inertia), float(icalc_floor),
                         (FLAG_BACKGROUND if background_update else 0) |
                         (FLAG_NEAR_FIELD if near_field is not None else 0) |
                         (FLAG_POSITIONS if max_shift is not None else 0),
                         float(max_shift) if max_shift is not None else 0.0)
        self.background = None
        nbytes = ctypes.c_size_t()
        check(lib().ptycho_workspace_bytes(ctypes.byref(self.desc), ctypes.byref(nbytes)))
        self.workspace_bytes = int(nbytes.value)
        if workspace is None:
            # torch's caching allocator returns 512-byte aligned blocks
            workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.device)
        if (workspace.dtype != torch.uint8 or workspace.numel() < self.workspace_bytes or
                workspace.device != self.device or workspace.data_ptr() % 256):
            raise ValueError("workspace must be a uint8 device tensor of at least workspace_bytes, "
                             "256-byte aligned")
        self.workspace = workspace
        self.iobs, self.mask, self.offsets = iobs, mask, offs
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib().ptycho_plan(ctypes.byref(self.desc), offs.ctypes.data, _ptr(iobs),
                                           _ptr(mask) if mask is not None else None,
                                           _ptr(self.workspace), self.workspace_bytes, stream,
                                           ctypes.byref(h)))
        self._h = h
        st = ctypes.c_int32()
        check(lib().ptycho_plan_stack(self._h, ctypes.byref(st)))
        self.stack = int(st.value)
        self.near_field = None
        if near_field is not None:
            self.set_near_field(near_field)

    @classmethod
    def with_positions(cls, pos_yx, iobs: torch.Tensor, mask: Optional[torch.Tensor], n_modes: int, obj_shape,
                       max_shift: float = 2.0, mult: float = 1.0, min_grad: float = 0.1, **kw) -> "Plan":
        """A plan on real (sub-pixel) scan positions that it refines on the
        device (positions within max_shift pixels of their start; see
        ptycho_plan_set_positions): windows from the positions, then the
        positions themselves."""
        offs, _ = windows_from_positions(pos_yx, int(iobs.shape[-1]), obj_shape)
        plan = cls(offs, iobs, mask, n_modes, obj_shape, max_shift=max_shift, **kw)
        plan.set_positions(pos_yx, mult, min_grad)
        return plan

    def set_positions(self, pos_yx, mult: float = 1.0, min_grad: float = 0.1) -> None:
        """Start (and current) positions of a plan created with max_shift, and
        the step factor and low-contrast filter of its position updates."""
        pos = np.ascontiguousarray(pos_yx, dtype=np.float64)
        if pos.shape != (self.j, 2):
            raise ValueError(f"positions must be [{self.j}][2]")
        with torch.cuda.device(self.device):
            self._enter()
            check(lib().ptycho_plan_set_positions(self._h, pos.ctypes.data, float(mult), float(min_grad)))

    def positions(self, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Device float64 [J][2]: the current positions (pixels from the object centre)."""
        out = torch.empty((self.j, 2), dtype=torch.float64, device=self.device) if out is None else out
        _need(out, "positions", torch.float64, (self.j, 2), self.device)
        self._enter()
        check(lib().ptycho_plan_positions(self._h, _ptr(out)))
        return out

    def refine(self, obj, probe, psi, shifts: Optional[torch.Tensor] = None):
        """One position-refinement step on the device from exit waves psi
        (shifts, update, new windows); `shifts` (float64 [J][3]) receives the
        shifts when given."""
        self._op(obj, probe)
        _need(psi, "psi", torch.complex64, (self.j, self.k, self.n, self.n), self.device)
        if shifts is not None:
            _need(shifts, "shifts", torch.float64, (self.j, 3), self.device)
        self._enter()
        check(lib().ptycho_refine_positions(self._h, _ptr(obj), _ptr(probe), _ptr(psi),
                                            _ptr(shifts) if shifts is not None else None))
        return shifts

    # -- helpers ---------------------------------------------------------
    def _enter(self):
        check(lib().ptycho_plan_set_stream(self._h, torch.cuda.current_stream(self.device).cuda_stream))

    def set_near_field(self, f) -> None:
        """Fresnel parameter(s) of a near-field plan: f or (f_y, f_x)."""
        fy, fx = (float(f), float(f)) if np.ndim(f) == 0 else (float(f[0]), float(f[1]))
        with torch.cuda.device(self.device):
            self._enter()
            check(lib().ptycho_plan_set_near_field(self._h, fy, fx))
        self.near_field = (fy, fx)

    def set_background(self, bg: Optional[torch.Tensor]) -> None:
        """Incoherent background float32 [N][N] (the detector layout of iobs) used by every later
        call, or None.  The plan keeps a reference; AP cycles with
        UPDATE_BACKGROUND refine it in place."""
        if bg is not None:
            _need(bg, "background", torch.float32, (self.n, self.n), self.device)
        check(lib().ptycho_plan_set_background(self._h, _ptr(bg) if bg is not None else None))
        self.background = bg

    def _op(self, obj, probe):
        _need(obj, "obj", torch.complex64, self.obj_shape, self.device)
        _need(probe, "probe", torch.complex64, (self.k, self.n, self.n), self.device)

    def close(self):
        if getattr(self, "_h", None):
            lib().ptycho_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points ----------------------------------------------------
    def ap_cycle(self, obj, probe, n_cycles: int = 1, update: int = 3, psi=None):
        """AP cycles.  `psi` (complex64 [J][K][N][N]) holds the projected exit
        waves; it is allocated here when the probe is updated and none is
        given."""
        self._op(obj, probe)
        if psi is None and (update & (_lib.UPDATE_PROBE | _lib.UPDATE_POSITIONS)):
            psi = torch.empty((self.j, self.k, self.n, self.n), dtype=torch.complex64, device=self.device)
        if psi is not None:
            _need(psi, "psi", torch.complex64, (self.j, self.k, self.n, self.n), self.device)
        self._enter()
        check(lib().ptycho_ap_cycle(self._h, _ptr(obj), _ptr(probe), _ptr(psi) if psi is not None else None,
                                    int(n_cycles), int(update)))
        return psi

    def dm_cycle(self, obj, probe, psi, n_cycles: int = 1, update: int = 3):
        self._op(obj, probe)
        _need(psi, "psi", torch.complex64, (self.j, self.k, self.n, self.n), self.device)
        self._enter()
        check(lib().ptycho_dm_cycle(self._h, _ptr(obj), _ptr(probe), _ptr(psi), int(n_cycles), int(update)))

    def psi_init(self, obj, probe, psi=None):
        self._op(obj, probe)
        if psi is None:
            psi = torch.empty((self.j, self.k, self.n, self.n), dtype=torch.complex64, device=self.device)
        _need(psi, "psi", torch.complex64, (self.j, self.k, self.n, self.n), self.device)
        self._enter()
        check(lib().ptycho_psi_init(self._h, _ptr(obj), _ptr(probe), _ptr(psi)))
        return psi

    LLK_MODELS = {"poisson": 0, "gaussian": 1, "euclidean": 2}

    def llk(self, obj, probe, out=None, model: str = "poisson"):
        """Device double[2]: (LLK sum, number of unmasked pixels) of the noise
        model `model` ("poisson", "gaussian" or "euclidean")."""
        self._op(obj, probe)
        if model not in self.LLK_MODELS:
            raise ValueError(f"unknown noise model {model!r}")
        out = torch.empty(2, dtype=torch.float64, device=self.device) if out is None else out
        self._enter()
        if model == "poisson":
            check(lib().ptycho_llk(self._h, _ptr(obj), _ptr(probe), _ptr(out)))
        else:
            check(lib().ptycho_llk_model(self._h, _ptr(obj), _ptr(probe), self.LLK_MODELS[model], _ptr(out)))
        return out

    def ml_grad(self, obj, probe, g_obj=None, g_probe=None, llk=None):
        self._op(obj, probe)
        g_obj = torch.empty_like(obj) if g_obj is None else g_obj
        g_probe = torch.empty_like(probe) if g_probe is None else g_probe
        _need(g_obj, "g_obj", torch.complex64, self.obj_shape, self.device)
        _need(g_probe, "g_probe", torch.complex64, (self.k, self.n, self.n), self.device)
        llk = torch.empty(2, dtype=torch.float64, device=self.device) if llk is None else llk
        self._enter()
        check(lib().ptycho_ml_grad(self._h, _ptr(obj), _ptr(probe), _ptr(g_obj), _ptr(g_probe), _ptr(llk)))
        return g_obj, g_probe, llk

    def ml_linesearch(self, obj, probe, d_obj, d_probe, out=None):
        self._op(obj, probe)
        _need(d_obj, "d_obj", torch.complex64, self.obj_shape, self.device)
        _need(d_probe, "d_probe", torch.complex64, (self.k, self.n, self.n), self.device)
        out = torch.empty(2, dtype=torch.float64, device=self.device) if out is None else out
        self._enter()
        check(lib().ptycho_ml_linesearch(self._h, _ptr(obj), _ptr(probe), _ptr(d_obj), _ptr(d_probe), _ptr(out)))
        return out

    def ml_state(self):
        nbytes = ctypes.c_size_t()
        check(lib().ptycho_ml_state_bytes(self._h, ctypes.byref(nbytes)))
        return torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)

    def ml_cycle(self, obj, probe, state, n_cycles: int = 1, update: int = 1, reset: bool = False,
                 hist: Optional[torch.Tensor] = None):
        self._op(obj, probe)
        if hist is not None:
            _need(hist, "hist", torch.float64, (int(n_cycles),), self.device)
        self._enter()
        check(lib().ptycho_ml_cycle(self._h, _ptr(obj), _ptr(probe), _ptr(state), int(n_cycles), int(update),
                                    1 if reset else 0, _ptr(hist) if hist is not None else None))

    TIMING_CLASSES = ("rows_fwd", "cols", "rows_inv", "gather_obj", "gather_probe", "probe_all",
                      "normalize", "other")

    def timing(self, enable: bool, classes=None):
        """Start (and reset) or stop per-kernel-class event timing; `classes`
        names the timed classes (TIMING_CLASSES), None = all."""
        mask = 0
        if enable:
            mask = 255 if classes is None else sum(1 << self.TIMING_CLASSES.index(c) for c in classes)
        check(lib().ptycho_plan_timing(self._h, mask))

    def timing_read(self):
        """{class: (total ms, launches)} since timing was last enabled."""
        out = {}
        for i, name in enumerate(self.TIMING_CLASSES):
            ms, n = ctypes.c_double(), ctypes.c_int64()
            check(lib().ptycho_plan_timing_read(self._h, i, ctypes.byref(ms), ctypes.byref(n)))
            out[name] = (float(ms.value), int(n.value))
        return out

    def position_shifts(self, obj, probe, psi, out=None):
        """Device double [J][3]: per frame (d_y, d_x, gradient energy) of the
        position refinement (Psi2PosShift) from exit waves psi."""
        self._op(obj, probe)
        _need(psi, "psi", torch.complex64, (self.j, self.k, self.n, self.n), self.device)
        out = torch.empty((self.j, 3), dtype=torch.float64, device=self.device) if out is None else out
        _need(out, "shifts", torch.float64, (self.j, 3), self.device)
        self._enter()
        check(lib().ptycho_position_shifts(self._h, _ptr(obj), _ptr(probe), _ptr(psi), _ptr(out)))
        return out

    def check_finite(self, obj, probe, out=None):
        """Device int32 [1]: 1 if the object or probe holds a NaN or inf."""
        self._op(obj, probe)
        out = torch.empty(1, dtype=torch.int32, device=self.device) if out is None else out
        _need(out, "flag", torch.int32, (1,), self.device)
        self._enter()
        check(lib().ptycho_check_finite(self._h, _ptr(obj), _ptr(probe), _ptr(out)))
        return out

    def rebuild(self, offsets) -> "Plan":
        """A plan on the same data, workspace and background with new frame
        offsets (after the positions moved).  This plan must not be used
        afterwards: the new one owns the workspace."""
        d = self.desc
        new = Plan(offsets, self.iobs, self.mask, self.k, self.obj_shape, stack=d.stack,
                   obj_inertia=d.obj_inertia, probe_inertia=d.probe_inertia, icalc_floor=d.icalc_floor,
                   workspace=self.workspace, background_update=bool(d.flags & FLAG_BACKGROUND),
                   near_field=self.near_field)
        if self.background is not None:
            new.set_background(self.background)
        self.close()
        return new

    def icalc(self, obj, probe, out=None):
        self._op(obj, probe)
        out = torch.empty((self.j, self.n, self.n), dtype=torch.float32, device=self.device) if out is None else out
        _need(out, "icalc", torch.float32, (self.j, self.n, self.n), self.device)
        self._enter()
        check(lib().ptycho_icalc(self._h, _ptr(obj), _ptr(probe), _ptr(out)))
        return out

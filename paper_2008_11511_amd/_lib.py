"""ctypes binding of libptycho.so (the C ABI in include/ptycho.h).

Argument marshalling only: every computation runs in the HIP library.  If
the library is missing or fails to load, `lib()` raises; nothing falls back
to another implementation.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libptycho.so")

OK = 0
STATUS = {0: "PTYCHO_OK", -1: "PTYCHO_E_INVALID", -2: "PTYCHO_E_BOUNDS",
          -3: "PTYCHO_E_UNSUPPORTED", -4: "PTYCHO_E_HIP", -5: "PTYCHO_E_WORKSPACE"}
UPDATE_OBJECT = 1
UPDATE_PROBE = 2
UPDATE_BACKGROUND = 4
UPDATE_POSITIONS = 8
FLAG_BACKGROUND = 1
FLAG_NEAR_FIELD = 2
FLAG_POSITIONS = 4


class PtychoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("n_frames", ctypes.c_int32), ("obj_ny", ctypes.c_int32),
                ("obj_nx", ctypes.c_int32), ("stack", ctypes.c_int32),
                ("obj_inertia", ctypes.c_float), ("probe_inertia", ctypes.c_float),
                ("icalc_floor", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("max_shift", ctypes.c_float)]


_P = ctypes.c_void_p
_SIGS = {
    "ptycho_offsets_from_positions": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "ptycho_windows_from_positions": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P],
    "ptycho_workspace_bytes": [ctypes.POINTER(Desc), ctypes.POINTER(ctypes.c_size_t)],
    "ptycho_plan": [ctypes.POINTER(Desc), _P, _P, _P, _P, ctypes.c_size_t, _P, ctypes.POINTER(_P)],
    "ptycho_plan_dry_run": [ctypes.POINTER(Desc), _P, ctypes.POINTER(ctypes.c_size_t)],
    "ptycho_plan_set_stream": [_P, _P],
    "ptycho_plan_set_background": [_P, _P],
    "ptycho_plan_set_near_field": [_P, ctypes.c_double, ctypes.c_double],
    "ptycho_position_shifts": [_P, _P, _P, _P, _P],
    "ptycho_update_positions": [ctypes.c_int32, _P, _P, _P, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P,
                                _P],
    "ptycho_plan_set_positions": [_P, _P, ctypes.c_double, ctypes.c_double],
    "ptycho_plan_positions": [_P, _P],
    "ptycho_refine_positions": [_P, _P, _P, _P, _P],
    "ptycho_check_finite": [_P, _P, _P, _P],
    "ptycho_plan_stack": [_P, ctypes.POINTER(ctypes.c_int32)],
    "ptycho_plan_destroy": [_P],
    "ptycho_ap_cycle": [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_uint32],
    "ptycho_dm_cycle": [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_uint32],
    "ptycho_psi_init": [_P, _P, _P, _P],
    "ptycho_llk": [_P, _P, _P, _P],
    "ptycho_llk_model": [_P, _P, _P, ctypes.c_int32, _P],
    "ptycho_ml_grad": [_P, _P, _P, _P, _P, _P],
    "ptycho_ml_linesearch": [_P, _P, _P, _P, _P, _P],
    "ptycho_ml_state_bytes": [_P, ctypes.POINTER(ctypes.c_size_t)],
    "ptycho_ml_cycle": [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_uint32, ctypes.c_int32, _P],
    "ptycho_llk_noalloc": [ctypes.POINTER(Desc), _P, _P, _P, _P, _P, _P, _P],
    "ptycho_icalc": [_P, _P, _P, _P],
    "ptycho_fft2": [ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int32, _P],
    "ptycho_plan_timing": [_P, ctypes.c_int32],
    "ptycho_plan_timing_read": [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "ptycho_last_error": [],
}

_lock = threading.Lock()
_lib = None


def lib() -> ctypes.CDLL:
    """Load libptycho.so (raises if it is missing or incomplete)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2008_11511_amd.build`")
            h = ctypes.CDLL(LIB_PATH)
            for name, args in _SIGS.items():
                fn = getattr(h, name)
                fn.argtypes = args
                fn.restype = ctypes.c_char_p if name == "ptycho_last_error" else ctypes.c_int
            _lib = h
        return _lib


def check(code: int) -> None:
    if code != OK:
        raise PtychoError(code, lib().ptycho_last_error().decode())


def exported_symbols():
    return list(_SIGS)

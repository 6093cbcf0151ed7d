"""MI355X (gfx950) ptychography hot path (far and near field).

The computation lives in the HIP library `libptycho.so` (C ABI in
include/ptycho.h).  This package only marshals torch tensors (device memory
and the current stream) into that ABI: `Plan` wraps a scan, `PoissonLLK` is
the autograd Function over the hand-written adjoint, and
`ReconstructionService` (module `serve`) runs on-line reconstructions
submitted as futures.
"""
from ._lib import PtychoError, UPDATE_BACKGROUND, UPDATE_OBJECT, UPDATE_POSITIONS, UPDATE_PROBE, lib  # noqa: F401
from .plan import Plan, offsets_from_positions, windows_from_positions, fft2  # noqa: F401
from .autograd import PoissonLLK, poisson_llk  # noqa: F401
from .serve import ReconstructionService  # noqa: F401

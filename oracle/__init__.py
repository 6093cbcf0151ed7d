"""FP64 CPU oracle for far- and near-field ptychography (test infrastructure only).

This package is the slow, plain reference that the GPU library is checked
against.  Only the tests, the smoke check and the CPU-baseline leg of the
benchmark may import it; the library itself never does, and this package
imports nothing from the library.
"""
from .ptycho import *  # noqa: F401,F403
from .ptycho import __all__  # noqa: F401

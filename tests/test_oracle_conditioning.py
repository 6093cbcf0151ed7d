"""Conditioning of one projection cycle, measured on the oracle alone.

From the AP/DM benchmark start (object = 1, probe = true probe with extra
defocus) almost every far-field pixel of the model is far below fp32
resolution while the data there hold photons, so the modulus projection
gives those pixels the phase of whatever is left: a relative input change at
the fp32 rounding level (6e-8) moves the FP64 oracle's own one-cycle output
by percents.  From a start near the truth the same change moves it by about
the same 1e-7.  This is why cycle parity with the fp32 GPU path is checked
from a start near the truth, and only the projected modulus from O = 1.
"""
import numpy as np

import oracle
import synth
from cases import make_problem, rel_l2


def _jitter(a, rng, eps=6e-8):
    return a * (1 + eps * (rng.standard_normal(a.shape) + 1j * rng.standard_normal(a.shape)))


def test_benchmark_start_is_ill_conditioned_near_truth_is_not():
    rng = np.random.default_rng(1)
    for start, lo, hi in (("apdm", 1e-3, 1.0), ("ml", 0.0, 1e-6)):
        pb = make_problem(synth.workload("ap64"), start=start)
        a = oracle.ap_cycle(pb.obj0, pb.probe0, pb.offsets, pb.iobs, pb.mask)
        b = oracle.ap_cycle(_jitter(pb.obj0, rng), _jitter(pb.probe0, rng), pb.offsets, pb.iobs, pb.mask)
        d = max(rel_l2(b[0], a[0]), rel_l2(b[1], a[1]))
        assert lo <= d <= hi, (start, d)

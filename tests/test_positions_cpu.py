"""Host side of the position update: the library's ptycho_update_positions
validates its arguments before enqueuing anything (no GPU needed), and the
oracle's update rule is pinned by hand-worked cases: the filter threshold
takes the median of an even count as the mean of the two middle values."""
import ctypes

import numpy as np

import oracle
from paper_2008_11511_amd import _lib


def test_update_positions_rejects_bad_arguments_before_gpu_work():
    h = _lib.lib()
    fake = ctypes.c_void_p(256)
    good = (fake, fake, fake, 1.0, 2.0, 0.1, fake, None)
    assert h.ptycho_update_positions(0, *good) == -1
    assert h.ptycho_update_positions(4, None, fake, fake, 1.0, 2.0, 0.1, fake, None) == -1
    assert h.ptycho_update_positions(4, fake, fake, fake, 1.0, 2.0, 0.1, None, None) == -1
    assert h.ptycho_update_positions(4, fake, fake, fake, 1.0, -1.0, 0.1, fake, None) == -1
    assert h.ptycho_update_positions(4, fake, fake, fake, float("nan"), 2.0, 0.1, fake, None) == -1
    assert h.ptycho_update_positions(4, fake, fake, fake, 1.0, 2.0, -0.5, fake, None) == -1
    assert h.ptycho_update_positions(4, fake, fake, fake, 1.0, float("inf"), 0.1, fake, None) == -1
    assert b"finite" in h.ptycho_last_error()


def test_update_filter_uses_the_mean_of_the_two_middle_energies():
    # energies 1, 2, 3, 10: median 2.5, threshold 0.5 * 2.5 = 1.25, so the
    # frame of energy 1 stays (with the lower middle value, 2, it would move)
    pos0 = np.zeros((4, 2))
    pos = np.zeros((4, 2))
    shifts = np.full((4, 2), 0.25)
    energy = np.array([1.0, 2.0, 3.0, 10.0])
    new = oracle.update_positions(pos, pos0, shifts, energy, mult=2.0, max_shift=2.0, min_grad=0.5)
    np.testing.assert_array_equal(new, [[0.0, 0.0], [0.5, 0.5], [0.5, 0.5], [0.5, 0.5]])
    # an odd count takes the middle value: energies 1, 2, 10 -> threshold 1.0 keeps all
    new3 = oracle.update_positions(pos[:3], pos0[:3], shifts[:3], np.array([1.0, 2.0, 10.0]), mult=2.0,
                                   max_shift=2.0, min_grad=0.5)
    np.testing.assert_array_equal(new3, np.full((3, 2), 0.5))

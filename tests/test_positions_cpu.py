"""Host side of the position refinement: the library's update rule against
the oracle's (same rule, independent code)."""
import numpy as np

import oracle
from paper_2008_11511_amd.plan import update_positions


def test_update_rule_matches_oracle():
    rng = np.random.default_rng(8)
    pos0 = rng.uniform(-50, 50, (200, 2))
    pos = pos0 + rng.uniform(-2.5, 2.5, (200, 2))
    shifts = rng.normal(0, 0.7, (200, 2))
    energy = rng.lognormal(0, 1.5, 200)
    for mult, mx, mg in ((1.0, 2.0, 0.1), (0.5, 1.0, 0.5), (2.0, 3.0, 0.0)):
        np.testing.assert_array_equal(update_positions(pos, pos0, shifts, energy, mult, mx, mg),
                                      oracle.update_positions(pos, pos0, shifts, energy, mult, mx, mg))

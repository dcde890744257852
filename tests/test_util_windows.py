"""The test helper that cuts one ghosted group out of a periodic box agrees
with the oracle's periodic ghost fill (so full-size parity tests can build
the oracle input of a few sampled groups without filling the whole box)."""
import numpy as np

import oracle as O
from tests._util import group_window


def test_group_window_equals_oracle_fill():
    rng = np.random.default_rng(4)
    box = rng.standard_normal((5, 32, 48, 16))
    for g in (2, 3, 4):
        want = O.fill_ghosts_periodic(box, g)
        for q in range(want.shape[0]):
            np.testing.assert_array_equal(group_window(box, q, g), want[q])

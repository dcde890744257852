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


def test_var_max_err_scales_each_variable():
    """An error in a momentum component that is small next to the energy is
    hidden by the one-scale measure and seen by the per-variable one."""
    import numpy as np
    from tests._util import scaled_max_err, var_max_err
    rng = np.random.default_rng(5)
    ref = np.empty((2, 5, 4, 4, 4))
    ref[:, 0] = 1 + rng.random((2, 4, 4, 4))
    ref[:, 1:4] = 1e-3 * rng.standard_normal((2, 3, 4, 4, 4))
    ref[:, 4] = 100 + rng.random((2, 4, 4, 4))
    got = ref.copy()
    got[:, 2] += 1e-12
    assert scaled_max_err(got, ref) < 1e-13
    assert var_max_err(got, ref) > 1e-10
    assert var_max_err(ref, ref) == 0.0

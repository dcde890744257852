"""The oracle's process pool over patch groups gives exactly the results of
solve_groups on the whole batch (the groups are independent; only the split
between processes differs)."""
import numpy as np

import oracle as O
from paper_1103_3373_amd import workloads as W


def test_group_pool_equals_serial():
    box = W.lognormal_blast_box(48, gamma=1.4, seed=5, radius_cells=3)
    G = O.fill_ghosts_periodic(box, 3)
    dt = O.cfl_dt(box, 1 / 48, 1.4, 0.5)
    want, _ = O.solve_groups(G, 3, dt, 1 / 48, 1.4, O.CTU, O.PPM, O.HLLC, O.VANLEER, O.F_CHAR)
    with O.GroupPool(3) as pool:
        got = pool.solve_groups(G, 3, dt, 1 / 48, 1.4, O.CTU, O.PPM, O.HLLC, O.VANLEER, O.F_CHAR)
    np.testing.assert_array_equal(got, want)

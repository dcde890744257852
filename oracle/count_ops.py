"""Count the floating-point operations of one cell update, per specialization.

Runs the op-counting build of the oracle (liboracle_count.so) on a periodic
box of smooth data, where every cell is updated exactly once and no ghost
ring is recomputed, and divides the counted operations (+ - * / sqrt and
comparisons; negation and absolute value are free sign operations) by the
number of cells.  This is the algorithmic work per cell update that the
benchmark's roofline uses.  Writes oracle/opcounts.json.

Test infrastructure: calls only the oracle.
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402


def smooth_box(n, gamma, seed=1):
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    f = [sum(rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + rng.uniform(0, 6.3))
             for k in rng.integers(-2, 3, size=(3, 3))) for _ in range(5)]
    rho = 1.0 + 0.1 * f[0]
    p = 1.0 + 0.1 * f[4]
    U = np.empty((5, n, n, n))
    U[0] = rho
    U[1], U[2], U[3] = rho * 0.1 * f[1], rho * 0.1 * f[2], rho * 0.1 * f[3]
    U[4] = p / (gamma - 1) + 0.5 * (U[1] ** 2 + U[2] ** 2 + U[3] ** 2) / rho
    return U


def count(scheme, recon, riemann, char, n=16, gamma=1.4):
    U = smooth_box(n, gamma)
    O.reset_ops()
    O.step_box(U, 1e-3, 1.0 / n, gamma, scheme, recon, riemann, 1, O.F_CHAR if char else 0, counting=True)
    return O.ops() / n ** 3


def main():
    names = {0: "MHM", 1: "VL", 2: "CTU"}
    rec = {0: "PLM", 1: "PPM"}
    rs = {0: "Roe", 1: "HLLC", 2: "HLLE"}
    out = {}
    for s in (0, 1, 2):
        for r in (0, 1):
            for q in (0, 1, 2):
                for c in (0, 1):
                    key = f"{names[s]}+{rec[r]}{'(char)' if c else ''}+{rs[q]}"
                    out[key] = round(count(s, r, q, c), 1)
                    print(key, out[key])
    with open(os.path.join(HERE, "opcounts.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()

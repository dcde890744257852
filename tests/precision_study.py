"""Precision study (run by hand on a GPU machine; not collected by pytest).

Kelvin-Helmholtz shear layer: the FP32 GPU path against the FP64 GPU path
and the FP64 oracle over 100 steps of MHM, VL and CTU (PPM(char) + HLLC) on
the oracle's time-step sequence, with the drift of the FP64 conserved sums;
then FP32 against FP64 on the GPU at a large size.  Prints one JSON line.

    python -m tests.precision_study [--n 64] [--big 512] [--steps 100]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def _rel(a, b):
    """Per-variable (L1, Linf) of a - b relative to b; the momentum components
    share the magnitude |m| of b as scale."""
    a = a.reshape(-1, 5, 4096).transpose(1, 0, 2).reshape(5, -1).astype(np.float64)
    b = b.reshape(-1, 5, 4096).transpose(1, 0, 2).reshape(5, -1).astype(np.float64)
    d = np.abs(a - b)
    mag = np.sqrt((b[1:4] ** 2).sum(0))
    s1 = np.array([np.abs(b[0]).sum()] + [mag.sum()] * 3 + [np.abs(b[4]).sum()])
    si = np.array([np.abs(b[0]).max()] + [mag.max()] * 3 + [np.abs(b[4]).max()])
    return (d.sum(1) / s1).tolist(), (d.max(1) / si).tolist()


def _drift(s, s0, mom):
    """Conserved-sum drift: relative for mass and energy, relative to the
    integral of |m| for the momenta."""
    scale = np.array([abs(s0[0]), mom, mom, mom, abs(s0[4])])
    return (np.abs(s - s0) / scale).tolist()


def precision_study(args):
    """Kelvin-Helmholtz shear layer: the FP32 GPU path against the FP64 GPU
    path and the FP64 oracle, 100 steps of MHM, VL and CTU (PPM(char) +
    HLLC) on the same time-step sequence, with FP64 conservation sums; and
    FP32 against FP64 on the GPU at the large size."""
    import torch
    from paper_1103_3373_amd import hydro as H
    from paper_1103_3373_amd import workloads as W

    gamma = 1.4
    res = {"metric": "precision study: rel L1 / Linf per conserved variable", "config": {}}
    n, steps = args.n, args.steps
    box = W.kelvin_helmholtz_box(n, gamma=gamma)
    grp = W.box_to_groups(box)
    import oracle as O
    for scheme, name, cfl in ((H.MHM, "MHM", 0.3), (H.VL, "VL", 0.3), (H.CTU, "CTU", 0.5)):
        print(f"[precision] {name} {n}^3 x {steps}", file=sys.stderr, flush=True)
        kw = dict(dh=1.0 / n, gamma=gamma, scheme=scheme, recon=H.PPM, riemann=H.HLLC, char=True)
        s64 = torch.from_numpy(grp).cuda()
        s32 = torch.from_numpy(grp.astype(np.float32)).cuda()
        o64, o32 = torch.empty_like(s64), torch.empty_like(s32)
        dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
        ref = box.copy()
        sums0 = H.conserved_sums(s64, 1.0 / n).cpu().numpy()
        mom = float(np.sqrt((grp[:, 1:4] ** 2).sum(1)).sum()) / n ** 3
        t_or = 0.0
        for _ in range(steps):
            dt = O.cfl_dt(ref, 1.0 / n, gamma, cfl)
            t1 = time.perf_counter()
            ref = O.step_box(ref, dt, 1.0 / n, gamma, scheme, H.PPM, H.HLLC, H.VANLEER, O.F_CHAR)
            t_or += time.perf_counter() - t1
            dt_dev.fill_(dt)
            H.step_box(s64, o64, (n, n, n), dt_dev, **kw)
            H.step_box(s32, o32, (n, n, n), dt_dev, **kw)
            s64, o64 = o64, s64
            s32, o32 = o32, s32
        torch.cuda.synchronize()
        g64, g32 = s64.cpu().numpy(), s32.cpu().numpy()
        refg = W.box_to_groups(ref)
        sums64 = H.conserved_sums(s64, 1.0 / n).cpu().numpy()
        sums32 = H.conserved_sums(s32, 1.0 / n).cpu().numpy()
        res[name] = {"fp32_vs_oracle": _rel(g32, refg), "fp64_vs_oracle": _rel(g64, refg),
                     "fp32_vs_fp64": _rel(g32, g64),
                     "sums_drift_fp64": _drift(sums64, sums0, mom),
                     "sums_drift_fp32": _drift(sums32, sums0, mom),
                     "oracle_s": t_or}
    N = args.big
    if N:
        print(f"[precision] {N}^3 FP32 vs FP64, CTU", file=sys.stderr, flush=True)
        big = W.box_to_groups(W.kelvin_helmholtz_box(N, gamma=gamma))
        kw = dict(dh=1.0 / N, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC, char=True)
        s64 = torch.from_numpy(big).cuda()
        mom = float(torch.sqrt((s64[:, 1:4] ** 2).sum(1)).sum()) / N ** 3
        del big
        s32 = s64.float()
        o64, o32 = torch.empty_like(s64), torch.empty_like(s32)
        dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
        sums0 = H.conserved_sums(s64, 1.0 / N).cpu().numpy()
        for _ in range(steps):
            H.cfl_dt(s64, 1.0 / N, gamma, 0.5, dt_out=dt_dev)
            H.step_box(s64, o64, (N, N, N), dt_dev, **kw)
            H.step_box(s32, o32, (N, N, N), dt_dev, **kw)
            s64, o64 = o64, s64
            s32, o32 = o32, s32
        torch.cuda.synchronize()
        sums64 = H.conserved_sums(s64, 1.0 / N).cpu().numpy()
        sums32 = H.conserved_sums(s32, 1.0 / N).cpu().numpy()
        l1, linf = [], []
        mag = torch.sqrt((s64[:, 1:4] ** 2).sum(1))
        for v in range(5):
            a = s32[:, v].double()
            b = s64[:, v]
            d = (a - b).abs()
            sc = mag if 1 <= v <= 3 else b.abs()
            l1.append((d.sum() / sc.sum()).item())
            linf.append((d.max() / sc.max()).item())
        del mag
        res[f"CTU_{N}"] = {"fp32_vs_fp64": (l1, linf),
                           "sums_drift_fp64": _drift(sums64, sums0, mom),
                           "sums_drift_fp32": _drift(sums32, sums0, mom)}
    res["config"] = {"workload": f"Kelvin-Helmholtz, {n}^3 x {steps} steps (GPU FP32, GPU FP64, oracle) and "
                                 f"{N}^3 x {steps} (GPU FP32 vs FP64), PPM(char, van Leer) + HLLC, gamma 1.4"}
    print(json.dumps(res))


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--n", type=int, default=64)
    p.add_argument("--big", type=int, default=512)
    p.add_argument("--steps", type=int, default=100)
    precision_study(p.parse_args())


if __name__ == "__main__":
    main()

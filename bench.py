"""Benchmark: cell updates per second of the unsplit CTU solver at 256^3.

Workload (one GPU): a 256^3 periodic box as 4096 patch groups of 16^3
interior cells, FP32, CTU + PPM (characteristic limiting, van Leer) + HLLC,
gamma = 1.4, seeded lognormal density with Mach-1 smooth velocities and 4
blasts (p = 100, r = 8 cells).

One step is the whole hot path, all on the device with the state resident
in HBM:
  a0-a8, a11  one persistent launch of the fused solver over the box: each
      group reads its 3 ghost layers straight from the neighbouring groups of
      the resident box (the preparation step fused into the solver), and the
      time step is read from device memory;
  a9, a10  FP64 CFL time step and FP64 conserved sums of the new state, in
      one pass over it (the time step is used by the next step).
Side measurements: the ghosted-groups API (periodic ghost fill, then the
solve), MHM and VL on the same box, a device copy for the bandwidth
reference, the plain per-group FP64 path on the same input for the speed-up,
and the oracle on a bounded sample of the same groups on the host cores.
Other modes: --amr (AMR-shaped batch with its preparation step), --serve
(continuous batching of a request stream).

Prints one JSON line.  Only the cpu_baseline leg imports the oracle.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-updates/s at 256^3 CTU+PPM+HLLC vs plain; HBM roofline %; p50/p99 step"
# Algorithmic floating-point operations per cell update of CTU + PPM(char) +
# HLLC, counted by the op-counting build of the oracle on a periodic box
# (no ghost-ring recomputation): + - * / sqrt and comparisons = 1, sign ops
# free.  Regenerate with oracle/count_ops.py.
OPS_PER_CELL = 2693.9
# The same count for the other schemes of the 256^3 workload (PPM(char) + HLLC).
OPS_PER_CELL_SCHEME = {"MHM": 1607.9, "VL": 1775.9, "CTU": OPS_PER_CELL}
# Published FP32 vector peak of MI355X: 256 CU x 4 SIMD x 16 lanes x 2 flop
# (FMA) x 2 (packed FP32) x 2.4 GHz = 157.3 TFLOP/s.  The kernels are built
# without packed FP32 instructions, so their own ceiling is half of it.
ALU_PEAK = 256 * 4 * 16 * 2 * 2 * 2.4e9
ALU_PEAK_NONPACKED = ALU_PEAK / 2
HBM_PEAK = 8.0e12
# Algorithmic HBM bytes per cell update of the box solver (FP32): read U^n and
# write U^{n+1} once each (5 x 4 B each way); ghost cells come from
# neighbouring groups of the same resident box.
BYTES_PER_CELL = 40.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--n", type=int, default=256, help="box size (multiple of 16)")
    p.add_argument("--plain-steps", type=int, default=2)
    p.add_argument("--cpu-seconds", type=float, default=8.0)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--extra-reps", type=int, default=10,
                   help="launches per side measurement (groups API, other schemes, copy); 0 skips them")
    p.add_argument("--no-autotune", action="store_true", help="skip the launch-shape autotuner")
    p.add_argument("--launch-shape", default=None, metavar="GRID,VARIANT,ZRUN",
                   help="pin the solver's launch shape instead of autotuning (hydro_set_launch_shape)")
    p.add_argument("--graph-replays", type=int, default=10, help="replays of a captured ten-step HIP graph")
    p.add_argument("--serve", action="store_true",
                   help="run the serving workload instead (Poisson arrivals, continuous batching)")
    p.add_argument("--amr", action="store_true",
                   help="run the AMR-shaped batched workload instead (3 levels, one persistent launch)")
    p.add_argument("--serve-requests", type=int, default=2000)
    p.add_argument("--serve-rate", type=float, default=200.0)
    p.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                   help="only run a device-to-device copy of MIB MiB three times (HBM counter calibration)")
    return p.parse_args()


def traffic_from_profile(kernel_src_hash: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "ctu_ppm_hllc_256_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_src_hash:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("csrc/fused_ctu.hpp", "csrc/fused_common.hpp", "csrc/hydro_math.hpp", "csrc/fused_ctu_f32.hip",
              "build.py"):
        with open(os.path.join(ROOT, "paper_1103_3373_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def host_cpu():
    """CPU model, logical CPUs and the CPUs this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(ghosted_dev, dt: float, dh: float, gamma: float, budget_s: float, box64_seed: int):
    """The FP64 oracle on the host cores, on the same first-step input as the
    GPU (CTU + PPM(char) + HLLC, ghosted groups copied to the host):
      * one thread on the leading groups until the time budget is used;
      * all usable cores (up to 16 worker processes, one share of the groups
        each: the analog of threading over patches) on every group;
      * one thread on whole 64^3 periodic boxes, 10 steps of MHM, VL and CTU
        (PPM(char) + HLLC, CFL 0.3 / 0.3 / 0.5), and the 32^3 Sod case of the
        plain path (MHM + PLM(primitive, van Leer) + Roe, gamma 5/3) in full,
        10 steps at CFL 0.5."""
    import oracle as O
    from paper_1103_3373_amd import workloads as W
    O._lib()
    model, ncpu, usable = host_cpu()
    workers = max(1, min(16, usable))
    total = ghosted_dev.shape[0]
    # One thread, bounded sample.
    t0 = time.perf_counter()
    done, el = 0, 0.0
    while done < total and el < budget_s:
        chunk = ghosted_dev[done:done + 32].cpu().numpy().astype(np.float64)
        for q in range(chunk.shape[0]):
            t1 = time.perf_counter()
            O.solve_groups(chunk[q:q + 1], 3, dt, dh, gamma, O.CTU, O.PPM, O.HLLC, O.VANLEER, O.F_CHAR)
            el += time.perf_counter() - t1
            done += 1
            if el >= budget_s:
                break
    one = done * 4096 / el
    # All usable cores, every group of the step.
    host = ghosted_dev.cpu().numpy()
    with O.GroupPool(workers) as pool:
        pool.solve_groups(host[:workers].astype(np.float64), 3, dt, dh, gamma, O.CTU, O.PPM, O.HLLC, O.VANLEER,
                          O.F_CHAR)  # workers started and warm
        t1 = time.perf_counter()
        pool.solve_groups(host.astype(np.float64), 3, dt, dh, gamma, O.CTU, O.PPM, O.HLLC, O.VANLEER, O.F_CHAR)
        el_all = time.perf_counter() - t1
    del host
    allc = total * 4096 / el_all
    # Whole 64^3 boxes, 10 steps per scheme, one thread.
    box64 = W.lognormal_blast_box(64, gamma=gamma, seed=box64_seed, radius_cells=2)
    per_scheme = {}
    for scheme, name, cfl in ((O.MHM, "MHM", 0.3), (O.VL, "VL", 0.3), (O.CTU, "CTU", 0.5)):
        st = box64.copy()
        t1 = time.perf_counter()
        for _ in range(10):
            st = O.step_box(st, O.cfl_dt(st, 1 / 64, gamma, cfl), 1 / 64, gamma, scheme, O.PPM, O.HLLC, O.VANLEER,
                            O.F_CHAR)
        per_scheme[name] = 10 * 64 ** 3 / (time.perf_counter() - t1)
    sod = W.sod_box(32, gamma=5.0 / 3.0)
    t1 = time.perf_counter()
    for _ in range(10):
        sod = O.step_box(sod, O.cfl_dt(sod, 1 / 32, 5.0 / 3.0, 0.5), 1 / 32, 5.0 / 3.0, O.MHM, O.PLM, O.ROE,
                         O.VANLEER, 0)
    c1 = 10 * 32 ** 3 / (time.perf_counter() - t1)
    return {"value": allc, "unit": "cell-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"all {total} patch groups of the same first-step input (CTU+PPM(char)+HLLC, FP64 oracle, "
                      f"g++ -O2) split over {workers} worker processes ({el_all:.1f} s); one thread: {done} groups "
                      f"in {el:.1f} s; whole 64^3 boxes x 10 steps per scheme and the 32^3 Sod case x 10 steps, "
                      f"one thread",
            "per_core_value": one, "cpu_model": model, "nproc": ncpu, "usable_cpus": usable,
            "box64_10_steps_one_thread": per_scheme, "sod32_mhm_plm_roe_fp64_one_thread": c1}


def amr_bench(args):
    """AMR-shaped step: 2048 + 6144 + 12288 patch groups (16^3 + 3 ghost
    cells) on three levels of refinement ratio 2 over a 256^3 base grid.
    Each timed step is the preparation step (every group's padded input from
    its own interior, the same-level groups that cover its ghost cells, and
    elsewhere the 64^3 coarse state blended between the start and the end of
    the coarse step at the level's sub-step time and interpolated
    trilinearly) and one persistent CTU + PPM(char) + Roe launch over all
    levels with fluxes on every group face (each level a segment with its own
    dh and dt scale); the launch shape comes from the autotuner.  The
    interiors start as trilinear interpolations of the coarse field; the
    coarse state at the end of the coarse step is that field advanced by one
    CTU step."""
    import torch
    from paper_1103_3373_amd import hydro as H
    from paper_1103_3373_amd import workloads as W

    gamma = 1.4
    counts = (2048, 6144, 12288)
    alpha = [0.5, 0.25, 0.875]  # fine sub-step times within the coarse step, per level
    n_total = sum(counts)
    g = H.ghost_width(H.CTU, H.PPM)
    dev = torch.device("cuda")
    cn = 64
    c0_box = W.amr_coarse_field(cn, gamma=gamma).astype(np.float32)
    coarse0 = torch.from_numpy(c0_box).to(dev)
    # Coarse state at the end of the coarse step: one CTU step of the 64^3 field.
    cg0 = torch.from_numpy(W.box_to_groups(c0_box)).to(dev)
    cg1 = torch.empty_like(cg0)
    cdt = torch.empty(1, dtype=torch.float64, device=dev)
    H.cfl_dt(cg0, 1.0 / cn, gamma, 0.5, dt_out=cdt)
    H.step_box(cg0, cg1, (cn, cn, cn), cdt, dh=1.0 / cn, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.ROE,
               char=True)
    coarse1 = torch.from_numpy(W.groups_to_box(cg1.cpu().numpy(), cn, cn, cn)).to(dev).contiguous()
    lay_np = W.amr_layout(counts, base_n=256)
    layout = torch.from_numpy(lay_np).to(dev)
    ng0 = 256 // 16
    gmap = H.build_group_map(layout, ng0, len(counts))
    groups = torch.empty((n_total, 5, 22, 22, 22), dtype=torch.float32, device=dev)
    out = torch.empty((n_total, 5, 16, 16, 16), dtype=torch.float32, device=dev)
    flux = torch.empty((n_total, 3, 2, 5, 16, 16), dtype=torch.float32, device=dev)
    dh0 = 1.0 / 256
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    H.fill_groups_interp(coarse0, layout, g, dh0, out=groups)
    # Interiors of the first step; the level-0 time step from all of them
    # (finer levels use dt / 2^l).
    out.copy_(groups[:, :, g:g + 16, g:g + 16, g:g + 16])
    H.cfl_dt(out, dh0, gamma, 0.5, dt_out=dt_dev)
    rows, first = [], 0
    for lev, cnt in enumerate(counts):
        sl = slice(first, first + cnt)
        rows.append((groups[sl], out[sl], flux[sl], dt_dev, 0.5 ** lev, dh0 * 0.5 ** lev, first, cnt))
        first += cnt
    table = H.seg_table(rows, dev)
    spec = H.make_spec(H.CTU, H.PPM, H.ROE, gamma=gamma, char=True)
    tuned = None if args.no_autotune else H.autotune(spec, n_total)
    stream = torch.cuda.current_stream()

    def prep():
        # The solve of the previous step left the interiors in `out`.
        H.fill_groups_amr(out, layout, gmap, ng0, alpha, coarse0, coarse1, g, out=groups)

    H.fill_groups_interp(coarse0, layout, g, dh0, out=groups)
    H.solve_batch(table, len(rows), n_total, spec)
    for _ in range(2):
        prep()
        H.solve_batch(table, len(rows), n_total, spec)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    fill_ms, solve_ms, interp_ms = [], [], []
    for _ in range(max(3, args.steps // 5)):
        ev[0].record(stream)
        prep()
        ev[1].record(stream)
        H.solve_batch(table, len(rows), n_total, spec)
        ev[2].record(stream)
        torch.cuda.synchronize()
        fill_ms.append(ev[0].elapsed_time(ev[1]))
        solve_ms.append(ev[1].elapsed_time(ev[2]))
    # For comparison: the whole padded groups interpolated from the coarse
    # field alone (no neighbours, one time).
    spare = torch.empty_like(groups)
    for _ in range(3):
        ev[0].record(stream)
        H.fill_groups_interp(coarse0, layout, g, dh0, out=spare)
        ev[1].record(stream)
        torch.cuda.synchronize()
        interp_ms.append(ev[0].elapsed_time(ev[1]))
    del spare
    # Coarse-grid correction at scale: the level-1 groups (6144 at 512^3, their
    # interiors and face fluxes from the solve above) refine a complete 256^3
    # coarse box, advanced by one CTU step with fluxes on every patch face.
    l1 = slice(counts[0], counts[0] + counts[1])
    cbox = torch.from_numpy(W.box_to_groups(W.lognormal_blast_box(256, gamma=gamma).astype(np.float32))).to(dev)
    cnew = torch.empty_like(cbox)
    cflux = torch.empty((cbox.shape[0], 3, 3, 5, 16, 16), dtype=torch.float32, device=dev)
    cdt = torch.empty(1, dtype=torch.float64, device=dev)
    H.cfl_dt(cbox, dh0, gamma, 0.5, dt_out=cdt)
    H.step_box(cbox, cnew, (256, 256, 256), cdt, dh=dh0, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.ROE,
               char=True, flux=cflux, flux_mid=True)
    cdt_h = float(cdt.item())
    flay = layout[l1].clone()
    flay[:, 0] = 0  # the fine level alone: its map has one level of 32 groups per side
    fmap = H.build_group_map(flay, 256 // 8, 1)
    assert int((fmap >= 0).sum().item()) == counts[1], "every level-1 group must be in the fine map"
    corr_ms = []
    for _ in range(5):
        work = cnew.clone()
        ev[0].record(stream)
        H.amr_correct(work, 256, cflux, out[l1], flay, fmap, flux[l1], cdt_h, dh0)
        ev[1].record(stream)
        torch.cuda.synchronize()
        corr_ms.append(ev[0].elapsed_time(ev[1]))
    corr_finite = bool(torch.isfinite(work).all().item())
    del cbox, cnew, cflux, work
    cells = n_total * 4096
    sm, fm = float(np.median(solve_ms)), float(np.median(fill_ms))
    d = H.get_diag(reset=True)
    out_json = {"metric": "AMR-shaped batched step: cell-updates/s, all levels in one persistent launch",
                "unit": "cell-updates/s", "value": cells / ((sm + fm) * 1e-3), "higher_is_better": True,
                "n_gpus": 1, "dtype": "f32",
                "data": "synthetic (interiors from the trilinear interpolation of a seeded 64^3 field; ghosts from "
                        "same-level neighbours or that field and its one-step successor, blended in time)",
                "config": {"workload": "levels of 2048/6144/12288 patch groups (16^3 + 3 ghosts) over a 256^3 "
                                       "base grid, CTU+PPM(char, van Leer)+Roe, fluxes on all group faces, one "
                                       "persistent launch", "alpha": alpha},
                "solve_ms": sm, "prep_ms": fm, "solve_cell_updates_per_s": cells / (sm * 1e-3),
                "coarse_only_interp_ms": float(np.median(interp_ms)),
                "correction_ms": float(np.median(corr_ms)), "correction_finite": corr_finite,
                "correction_workload": "refluxing + restriction: 6144 level-1 groups (512^3 grid) over a complete "
                                       "256^3 coarse box",
                "autotune_grid": tuned, "roe_fallbacks": d["roe_fallbacks"], "floor_hits": d["floor_hits"],
                "finite": bool(torch.isfinite(out).all().item())}
    print(json.dumps(out_json))


def serve_bench(args):
    """Serving workload: Poisson arrivals (mean 200/s) of independent
    simulations, box 32^3/64^3/128^3, MHM/VL/CTU, Roe/HLLC, Sod/blast/
    lognormal initial conditions, PPM (characteristic, van Leer), FP32, 50
    steps each, admission by footprint under 200 GB.  Initial states are
    drawn from 4 seeded variants per (IC, size), generated before the run."""
    import torch
    from paper_1103_3373_amd import workloads as W
    from paper_1103_3373_amd.serve import GpuBackend, Request, Server

    gamma = 1.4
    stream = W.request_stream(n_requests=args.serve_requests, rate=args.serve_rate)
    reqs = [Request(r["id"], r["arrival"], r["n"], r["scheme"], r["riemann"], r["ic"], r["seed"] % 4, 50)
            for r in stream]
    cache = {}
    print(f"[serve] generating initial states", file=sys.stderr, flush=True)
    reports = {}
    for overlap in (False, True):
        be = GpuBackend(gamma=gamma, ic_cache=cache, overlap=overlap)
        for ic in ("sod", "blast", "lognormal"):
            for n in (32, 64, 128):
                for seed in range(4):
                    be._ic(Request(0, 0.0, n, 0, 0, ic, seed))
        # Warm-up: every specialization once at the largest size (one-time
        # kernel attributes and scratch growth happen here, not in the timed run).
        print(f"[serve] warm-up (overlap={overlap})", file=sys.stderr, flush=True)
        warm = Server(be)
        k = 0
        for s in (0, 1, 2):
            for rs in (0, 1):
                for _ in range(8):
                    warm.submit(Request(10 ** 6 + k, 0.0, 128, s, rs, "lognormal", 0, 2))
                    k += 1
        warm.run()
        torch.cuda.synchronize()
        print(f"[serve] {len(reqs)} requests at {args.serve_rate}/s (overlap={overlap})", file=sys.stderr, flush=True)
        srv = Server(be, mem_cap=200e9)
        for r in reqs:
            srv.submit(r)
        srv.run()
        reports[overlap] = dict(srv.report(), table_uploads=be.table_builds)
    rep = reports[True]
    offered = sum(r.n ** 3 * r.steps for r in reqs) / (reqs[-1].arrival if reqs else 1.0)
    out = {"metric": "serving: p50/p99 per-step latency and aggregate cell-updates/s", "unit": "cell-updates/s",
           "value": rep["cell_updates_per_s"], "higher_is_better": True, "n_gpus": 1, "dtype": "f32",
           "data": "synthetic (Sod / blast / lognormal seeded initial conditions)",
           "config": {"workload": f"{len(reqs)} Poisson requests, mean {args.serve_rate}/s, boxes 32^3/64^3/128^3, "
                                  "MHM/VL/CTU x Roe/HLLC, PPM(char, van Leer), 50 steps, 200 GB cap",
                      "backend": "one stream per scheme, resident segment tables"},
           "offered_cell_updates_per_s": offered, **rep,
           "single_stream": reports[False]}
    print(json.dumps(out))


def _time_launches(fn, reps, stream):
    """Mean ms of `reps` back-to-back calls of fn, HIP events on `stream`."""
    import torch
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def side_measurements(args, H, W, state, nxt, dt_dev, n, gamma, dh, stream):
    """Measurements beside the headline step, outside its timed region:
    the ghosted-groups API (ghost fill a0 + solve) on the same state, the
    box-API solve of MHM and VL at the same size, and a device copy for the
    measured HBM bandwidth."""
    import torch
    reps = args.extra_reps
    cells = n ** 3
    G = (n // 16) ** 3
    print(f"[bench] side measurements, {reps} launches each", file=sys.stderr, flush=True)
    res = {"reps": reps}
    g = H.ghost_width(H.CTU, H.PPM)
    ghosted = torch.empty((G, 5, 16 + 2 * g, 16 + 2 * g, 16 + 2 * g), dtype=torch.float32, device=state.device)
    kw = dict(dh=dh, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC, limiter=H.VANLEER, char=True)
    fill_ms = _time_launches(lambda: H.fill_ghosts_periodic(state, g, grouped=True, shape=(n, n, n), out=ghosted),
                             reps, stream)
    dt = float(dt_dev.item())
    solve_ms = _time_launches(lambda: H.solve_groups(ghosted, nxt, None, dt=dt, **kw), reps, stream)
    res["groups_api_CTU"] = {"fill_ms": fill_ms, "solve_ms": solve_ms,
                             "cell_updates_per_s_with_fill": cells / ((fill_ms + solve_ms) * 1e-3),
                             "cell_updates_per_s_without_fill": cells / (solve_ms * 1e-3),
                             "algorithmic_bytes_per_cell": 72.0}
    del ghosted
    for name, scheme in (("MHM", H.MHM), ("VL", H.VL)):
        kws = dict(kw, scheme=scheme)
        ms = _time_launches(lambda: H.step_box(state, nxt, (n, n, n), dt_dev, dt_scale=0.6, **kws), reps, stream)
        ops = OPS_PER_CELL_SCHEME[name]
        res[f"box_api_{name}"] = {"solve_ms": ms, "cell_updates_per_s": cells / (ms * 1e-3),
                                  "ops_per_cell": ops, "alu_frac": ops * cells / (ms * 1e-3) / ALU_PEAK}
    a = torch.empty(1 << 28, dtype=torch.float32, device=state.device)  # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    cms = _time_launches(lambda: b.copy_(a), reps, stream)
    res["copy_GBps"] = 2 * a.numel() * 4 / (cms * 1e-3) / 1e9
    del a, b
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the solver library has no multi-GPU "
              "path; patch groups would shard by domain decomposition with a halo exchange.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1103_3373_amd import hydro as H
    from paper_1103_3373_amd import workloads as W

    if args.copy_calibration:
        nb = args.copy_calibration << 20
        a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nb, "copy_bytes_written": nb, "launches": 3}))
        return

    if args.serve:
        serve_bench(args)
        return
    if args.amr:
        amr_bench(args)
        return

    n = args.n
    gamma, dh, cfl = 1.4, 1.0 / n, 0.5
    G = (n // 16) ** 3
    cells = n ** 3
    dev = torch.device("cuda")
    print(f"[bench] generating {n}^3 lognormal+blast input", file=sys.stderr, flush=True)
    box = W.lognormal_blast_box(n, gamma=gamma, seed=W.IC_SEED)
    state = torch.from_numpy(W.box_to_groups(box).astype(np.float32)).to(dev)
    nxt = torch.empty_like(state)
    g = H.ghost_width(H.CTU, H.PPM)
    dt_dev = torch.empty(1, dtype=torch.float64, device=dev)
    sums = torch.empty(5, dtype=torch.float64, device=dev)
    spec = H.make_spec(H.CTU, H.PPM, H.HLLC, H.VANLEER, gamma=gamma, char=True)
    tuned = None
    if args.launch_shape:
        gr, var, zr = (int(v) for v in args.launch_shape.split(","))
        H.set_launch_shape(spec, gr, var, zr)
        tuned = f"pinned {gr},{var},{zr}"
    elif not args.no_autotune:
        tuned = H.autotune(spec, G)
        print(f"[bench] autotune: grid {tuned}", file=sys.stderr, flush=True)
    shape = H.get_launch_shape(spec, (n, n, n))
    print(f"[bench] launch shape (grid, variant, zrun): {shape}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    solve_kw = dict(dh=dh, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC, limiter=H.VANLEER, char=True)

    H.cfl_dt(state, dh, gamma, cfl, dt_out=dt_dev)
    torch.cuda.synchronize()
    dt0 = dt_dev.item()

    k_ev = []  # (start, end) events around every solver launch in the timed region

    def step(i, record):
        src, dst = (state, nxt) if i % 2 == 0 else (nxt, state)
        if record:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        # a0 + a1-a8 (+ a11): the fused solver reads the ghost cells from the
        # resident box and is launched persistently over all groups.
        H.step_box(src, dst, (n, n, n), dt_dev, **solve_kw)
        if record:
            e1.record(stream)
            k_ev.append((e0, e1))
        H.cfl_dt_sums(dst, dh, gamma, cfl, dt_out=dt_dev, sums_out=sums)  # a9 + a10, one pass

    print(f"[bench] warmup {args.warmup} steps", file=sys.stderr, flush=True)
    for i in range(args.warmup):
        step(i, False)
    torch.cuda.synchronize()
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    print(f"[bench] timing {args.steps} steps", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_ev[0].record(stream)
    for i in range(args.steps):
        step(args.warmup + i, True)
        step_ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps)])  # ms
    # The same steps replayed from a captured HIP graph (ten steps per graph,
    # an even count so the double buffers end where they started).
    graph_ms = None
    graph_steps = 10
    if args.graph_replays > 0:
        side = torch.cuda.Stream()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            for i in range(graph_steps):
                step(i, False)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        g0, g1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        g0.record(stream)
        for _ in range(args.graph_replays):
            graph.replay()
        g1.record(stream)
        torch.cuda.synchronize()
        graph_ms = g0.elapsed_time(g1) / (graph_steps * args.graph_replays)
    total_ms = step_ev[0].elapsed_time(step_ev[-1])
    kern_ms = np.array([a.elapsed_time(b) for a, b in k_ev])
    ms_per_step = total_ms / args.steps
    value = cells / (ms_per_step * 1e-3)
    kern_avg = float(kern_ms.mean())
    achieved = OPS_PER_CELL * cells / (kern_avg * 1e-3)
    final_dt = dt_dev.item()
    final_sums = sums.cpu().numpy().tolist()
    assert np.isfinite(final_dt) and final_dt > 0, final_dt

    extras = side_measurements(args, H, W, state, nxt, dt_dev, n, gamma, dh, stream) if args.extra_reps > 0 else None

    # Plain per-group FP64 path on the same first-step input (solver only).
    plain = None
    if not args.no_plain and args.plain_steps > 0:
        print(f"[bench] plain FP64 path, {args.plain_steps} launches", file=sys.stderr, flush=True)
        st64 = torch.from_numpy(W.box_to_groups(box)).to(dev)
        gh64 = H.fill_ghosts_periodic(st64, g, grouped=True, shape=(n, n, n))  # plain path needs ghosted groups
        del st64
        out64 = torch.empty((G, 5, 16, 16, 16), dtype=torch.float64, device=dev)
        H.solve_groups(gh64, out64, None, dt=dt0, dh=dh, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC,
                       limiter=H.VANLEER, char=True, plain=True)
        torch.cuda.synchronize()
        pe = [torch.cuda.Event(enable_timing=True) for _ in range(args.plain_steps + 1)]
        pe[0].record(stream)
        for i in range(args.plain_steps):
            H.solve_groups(gh64, out64, None, dt=dt0, dh=dh, gamma=gamma, scheme=H.CTU, recon=H.PPM,
                           riemann=H.HLLC, limiter=H.VANLEER, char=True, plain=True)
            pe[i + 1].record(stream)
        torch.cuda.synchronize()
        pms = pe[0].elapsed_time(pe[-1]) / args.plain_steps
        plain = {"path": "plain per-group FP64 (one workgroup per group, global temporaries)",
                 "ms_per_solve": round(pms, 3), "cell_updates_per_s": cells / (pms * 1e-3),
                 "speedup_of_fused_solve": round(pms / kern_avg, 2)}
        # The exact Riemann solver (plain path only) on the same input, FP64.
        H.get_diag(reset=True)
        pe[0].record(stream)
        H.solve_groups(gh64, out64, None, dt=dt0, dh=dh, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.EXACT,
                       limiter=H.VANLEER, char=True)
        pe[1].record(stream)
        torch.cuda.synchronize()
        ems = pe[0].elapsed_time(pe[1])
        plain["exact_solver"] = {"ms_per_solve": round(ems, 3), "cell_updates_per_s": cells / (ems * 1e-3),
                                 "vacuum_or_unconverged_faces": H.get_diag(reset=True)["roe_fallbacks"],
                                 "finite": bool(torch.isfinite(out64).all().item())}
        del gh64, out64

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] oracle CPU baseline", file=sys.stderr, flush=True)
        first = torch.from_numpy(W.box_to_groups(box).astype(np.float32)).to(dev)
        ghosted = H.fill_ghosts_periodic(first, g, grouped=True, shape=(n, n, n))
        del first
        torch.cuda.synchronize()
        cpu = cpu_baseline(ghosted, dt0, dh, gamma, args.cpu_seconds, W.IC_SEED)
        del ghosted

    src_hash = kernel_source_hash()
    traffic = traffic_from_profile(src_hash)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded lognormal density, Mach-1 smooth velocities, 4 blasts p=100 r=8)",
        "config": {"workload": f"{n}^3 periodic box, {G} patch groups of 16^3 + 3 ghost cells, CTU+PPM(char, van "
                               f"Leer)+HLLC, gamma 1.4, CFL 0.5", "n_groups": G, "ghost": g,
                   "step": "fused box solve (ghosts read from the resident box) + FP64 dt and sums (one pass)"},
        "p50_step_ms": float(np.percentile(per_step, 50)),
        "graph_ms_per_step": graph_ms,
        "p99_step_ms": float(np.percentile(per_step, 99)),
        "wall_s": wall,
        "solver_kernel_ms": kern_avg,
        "solver_cell_updates_per_s": cells / (kern_avg * 1e-3),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": ALU_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / ALU_PEAK, "traffic": traffic,
                     "peak_nonpacked": ALU_PEAK_NONPACKED / 1e12, "frac_of_nonpacked": achieved / ALU_PEAK_NONPACKED,
                     "ops_per_cell": OPS_PER_CELL, "kernel": "ctu_fused_kernel<float, PPM, HLLC>",
                     "kernel_source_sha256": src_hash},
        "hbm": {"algorithmic_bytes_per_cell": BYTES_PER_CELL,
                "algorithmic_GBps": BYTES_PER_CELL * cells / (kern_avg * 1e-3) / 1e9,
                "frac_of_8TBps": BYTES_PER_CELL * cells / (kern_avg * 1e-3) / HBM_PEAK},
        "plain": plain,
        "side": extras,
        "cpu_baseline": cpu,
        "autotune_grid": tuned,
        "launch_shape": {"grid": shape[0], "variant": shape[1], "zrun": shape[2]},
        "final_dt": final_dt,
        "final_sums": final_sums,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

"""GPU tests of the batched / box / graph paths (through the C ABI).

* The box step (ghost cells read from the resident grouped box) equals the
  ghost fill followed by the groups solve bit for bit, and the oracle.
* One persistent launch over uneven AMR-shaped levels (segments with their
  own cell size and time-step scale) equals separate per-level launches bit
  for bit, face fluxes included, and the oracle.
* A captured HIP graph of whole steps, replayed several times with eager
  work in between, reproduces the eager results bit for bit.
* Results do not depend on the launch shape chosen by the autotuner.
"""
import numpy as np
import pytest

import oracle as O
from paper_1103_3373_amd import workloads as W
from tests._util import rel_errors, random_smooth_box, scaled_max_err, var_max_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1103_3373_amd import hydro
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    hydro.lib()
    return hydro


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _max_rel_per_var(a, b):
    """max |a - b| over each variable's cells / max |b| of that variable."""
    a = a.double().transpose(0, 1).reshape(5, -1)
    b = b.double().transpose(0, 1).reshape(5, -1)
    return ((a - b).abs().max(1).values / b.abs().max(1).values).max().item()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("scheme,recon,rs", [(2, 1, 1), (2, 0, 0), (2, 1, 2), (0, 1, 1), (0, 0, 1), (1, 1, 1),
                                             (1, 1, 0)])
def test_box_zruns_match_groups_path(H, dtype, scheme, recon, rs):
    """A box step without flux output marches through runs of z-consecutive
    groups (tile depth 16 * zrun; for VL, its second stage).  With one group
    per run, CTU and MHM equal the ghosted-groups path (which marches each
    group alone) bit for bit; VL's box predictor computes the half step once
    per cell with an instantiation of its own, which may contract FMAs
    differently from the ghosted one, so VL agrees to a few ulps.  With longer
    runs, the first planes of a group that continues a run take their z
    slopes and edges from the loop body instead of the kernel's z prologue,
    two inlined copies of the same arithmetic whose multiply-adds the
    compiler may fuse differently, so they agree to the parity bars (relative
    to each variable's maximum: 1e-12 in FP64, 1e-5 in FP32), and bit for bit
    across workgroup counts at one run length.  Requests include lengths that
    are not built (8 -> 4) or do not divide the box's 8 groups in z (3 -> 2);
    FP64, and MHM / VL with PLM, have one group per run only."""
    gamma = 1.4
    nx, ny, nz = 32, 16, 128
    big = W.lognormal_blast_box(128, gamma=gamma, seed=29, radius_cells=4)
    box = big[:, :nz, :ny, :nx].copy()
    grouped = _dev(W.box_to_groups(box), dtype)
    g = H.ghost_width(scheme, recon)
    dt = O.cfl_dt(box, 1 / 128, gamma, 0.5 if scheme == 2 else 0.3)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
    ghosted = H.fill_ghosts_periodic(grouped, g, grouped=True, shape=(nx, ny, nz))
    ref = torch.empty_like(grouped)
    H.solve_groups(ghosted, ref, None, dt=dt, dh=1 / 128, gamma=gamma, scheme=scheme, recon=recon, riemann=rs,
                   char=True)
    f64 = dtype == torch.float64
    spec = H.make_spec(scheme, recon, rs, H.VANLEER, gamma=gamma, char=True, f64=f64)
    variant = 2 if f64 else 4
    bar = 1e-12 if f64 else 1e-5
    ulps = 4 * (2.0 ** -52 if f64 else 2.0 ** -23)
    by_run = {}
    try:
        for zrun, grid in ((1, 0), (1, 5), (2, 0), (4, 7), (8, 3), (8, 0), (3, 5), (0, 0)):
            H.set_launch_shape(spec, grid, variant, zrun)
            used = H.get_launch_shape(spec, (nx, ny, nz))[2]
            out = torch.empty_like(grouped)
            H.step_box(grouped, out, (nx, ny, nz), dt_dev, dh=1 / 128, gamma=gamma, scheme=scheme, recon=recon,
                       riemann=rs, char=True)
            torch.cuda.synchronize()
            assert torch.isfinite(out).all().item()
            if used == 1 and scheme != 1:
                assert torch.equal(out, ref), (zrun, grid)
            elif used == 1:
                assert ((out - ref).abs().max() / ref.abs().max()).item() <= ulps, (zrun, grid)
            else:
                assert _max_rel_per_var(out, ref) <= bar, (zrun, grid)
            if used in by_run:
                assert torch.equal(out, by_run[used]), (zrun, grid)
            by_run[used] = out
        built = not f64 and (scheme == 2 or recon == 1)
        assert sorted(by_run) == ([1, 2, 4] if built else [1])
    finally:
        H.set_launch_shape(spec, 0, variant, 0)


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("recon,rs,char", [(1, 1, True), (1, 0, False), (0, 2, True), (0, 1, False)])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_step_box_equals_fill_and_solve(H, scheme, recon, rs, char, dtype):
    gamma = 1.4
    nx, ny, nz = 48, 32, 16
    box = W.lognormal_blast_box(48, gamma=gamma, seed=13, radius_cells=4)[:, :nz, :ny, :nx].copy()
    grouped = _dev(W.box_to_groups(box), dtype)
    G = grouped.shape[0]
    g = H.ghost_width(scheme, recon)
    dt = O.cfl_dt(box, 1 / 48, gamma, 0.4 if scheme == 2 else 0.3)
    dt_dev = torch.tensor([dt], dtype=torch.float64, device="cuda")
    out_box = torch.empty_like(grouped)
    fl_box = torch.empty((G, 3, 3, 5, 16, 16), dtype=dtype, device="cuda")
    H.step_box(grouped, out_box, (nx, ny, nz), dt_dev, dh=1 / 48, gamma=gamma, scheme=scheme, recon=recon,
               riemann=rs, char=char, flux=fl_box, flux_mid=True)
    ghosted = H.fill_ghosts_periodic(grouped, g, grouped=True, shape=(nx, ny, nz))
    out_ref = torch.empty_like(grouped)
    fl_ref = torch.empty_like(fl_box)
    H.solve_groups(ghosted, out_ref, fl_ref, dt=dt, dh=1 / 48, gamma=gamma, scheme=scheme, recon=recon, riemann=rs,
                   char=char, flux_mid=True)
    torch.cuda.synchronize()
    if scheme == 1:
        # The box path computes the VL half step once per cell with the
        # interiors-only predictor (a different kernel instantiation, whose
        # compiled FMA contractions may differ in the last bit); the groups
        # path uses the ghosted one.  Hold them to a few ulps.
        tol = 4 * (2.0 ** -23 if dtype == torch.float32 else 2.0 ** -52)
        scale = out_ref.abs().max()
        assert ((out_box - out_ref).abs().max() / scale).item() <= tol
        assert ((fl_box - fl_ref).abs().max() / fl_ref.abs().max()).item() <= tol
    else:
        assert torch.equal(out_box, out_ref)
        assert torch.equal(fl_box, fl_ref)
    # and the oracle on the whole periodic box
    src = W.box_to_groups(box) if dtype == torch.float64 else W.box_to_groups(box).astype(np.float32)
    ref = O.step_box(W.groups_to_box(src.astype(np.float64), nx, ny, nz), dt, 1 / 48, gamma, scheme, recon, rs, 1,
                     O.F_CHAR if char else 0)
    got = W.groups_to_box(out_box.cpu().numpy().astype(np.float64), nx, ny, nz)
    if dtype == torch.float64:
        assert scaled_max_err(got, ref) <= 1e-12
        assert var_max_err(got, ref) <= 1e-12
    else:
        l1, _ = rel_errors(got, ref)
        assert l1.max() <= 1e-5


def test_amr_levels_in_one_launch(H):
    """Three levels with different cell sizes and dt scales (refinement ratio
    2) as segments of one persistent launch == per-level launches; the
    preparation step is the trilinear fill from a coarse field."""
    gamma = 1.4
    coarse = W.amr_coarse_field(32, gamma=gamma, seed=21)
    counts = (7, 12, 20)
    lay = W.amr_layout(counts, base_n=64, seed=21)
    g = 3
    dev_coarse = _dev(coarse, torch.float32)
    G = H.fill_groups_interp(dev_coarse, torch.from_numpy(lay).cuda(), g, 1 / 64)
    n = G.shape[0]
    out = torch.empty((n, 5, 16, 16, 16), dtype=torch.float32, device="cuda")
    flux = torch.empty((n, 3, 2, 5, 16, 16), dtype=torch.float32, device="cuda")
    dt0 = 0.25 * (1 / 64) / 4.0
    dt_dev = torch.tensor([dt0], dtype=torch.float64, device="cuda")
    segs, first = [], 0
    for lev, cnt in enumerate(counts):
        sl = slice(first, first + cnt)
        segs.append((G[sl], out[sl], flux[sl], dt_dev, 0.5 ** lev, (1 / 64) * 0.5 ** lev, first, cnt))
        first += cnt
    spec = H.make_spec(H.CTU, H.PPM, H.ROE, gamma=gamma, char=True)
    table = H.seg_table(segs, "cuda")
    H.solve_batch(table, len(segs), n, spec)
    torch.cuda.synchronize()
    ref_out = torch.empty_like(out)
    ref_flux = torch.empty_like(flux)
    first = 0
    for lev, cnt in enumerate(counts):
        sl = slice(first, first + cnt)
        H.solve_groups(G[sl], ref_out[sl], ref_flux[sl], dt=dt0 * 0.5 ** lev, dh=(1 / 64) * 0.5 ** lev,
                       gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.ROE, char=True)
        first += cnt
    torch.cuda.synchronize()
    assert torch.equal(out, ref_out)
    assert torch.equal(flux, ref_flux)
    # oracle on a few groups of each level (FP64 on the same FP32 inputs)
    Gh = G.cpu().numpy().astype(np.float64)
    first = 0
    for lev, cnt in enumerate(counts):
        pick = [first, first + cnt - 1]
        ref, rfl = O.solve_groups(Gh[pick], g, dt0 * 0.5 ** lev, (1 / 64) * 0.5 ** lev, gamma, 2, 1, 0, 1, O.F_CHAR,
                                  want_flux=True)
        l1, _ = rel_errors(out[pick].cpu().numpy(), ref)
        assert l1.max() <= 1e-5
        assert scaled_max_err(flux[pick].cpu().numpy(), rfl) <= 1e-5
        first += cnt


def test_graph_replay_matches_eager(H):
    gamma = 1.4
    n = 64
    box = W.lognormal_blast_box(n, gamma=gamma, seed=5)
    s0 = _dev(W.box_to_groups(box), torch.float32)
    a, b = s0.clone(), torch.empty_like(s0)
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    sums = torch.empty(5, dtype=torch.float64, device="cuda")
    kw = dict(dh=1 / n, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC, char=True)

    def two_steps():
        H.step_box(a, b, (n, n, n), dt_dev, **kw)
        H.cfl_dt(b, 1 / n, gamma, 0.5, dt_out=dt_dev)
        H.step_box(b, a, (n, n, n), dt_dev, **kw)
        H.cfl_dt(a, 1 / n, gamma, 0.5, dt_out=dt_dev)
        H.conserved_sums(a, 1 / n, sums_out=sums)

    # eager reference: 3 x two steps
    a.copy_(s0)
    H.cfl_dt(a, 1 / n, gamma, 0.5, dt_out=dt_dev)
    eager = []
    for _ in range(3):
        two_steps()
        torch.cuda.synchronize()
        eager.append((a.clone(), dt_dev.clone(), sums.clone()))
    # capture (after a warm-up that performs one-time setup)
    a.copy_(s0)
    H.cfl_dt(a, 1 / n, gamma, 0.5, dt_out=dt_dev)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        two_steps()
    a.copy_(s0)
    H.cfl_dt(a, 1 / n, gamma, 0.5, dt_out=dt_dev)
    torch.cuda.synchronize()
    for r in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(a, eager[r][0]), r
        assert torch.equal(dt_dev, eager[r][1]), r
        assert torch.equal(sums, eager[r][2]), r
        _ = (a.float().sum() * 0).item()  # eager work between replays


def test_launch_shape_does_not_change_results(H):
    gamma = 1.4
    box = random_smooth_box(64, gamma, 8, amp=0.3)
    g = 3
    G = H.fill_ghosts_periodic(_dev(box, torch.float32), g)
    kw = dict(dt=2e-3, dh=1 / 64, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC, char=True)
    o1 = torch.empty((G.shape[0], 5, 16, 16, 16), device="cuda")
    H.solve_groups(G, o1, None, **kw)
    best = H.autotune(H.make_spec(H.CTU, H.PPM, H.HLLC, gamma=gamma, char=True), G.shape[0])
    assert best > 0
    o2 = torch.empty_like(o1)
    H.solve_groups(G, o2, None, **kw)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("recon,riemann", [(1, 1), (1, 0), (0, 2)])
def test_every_launch_variant_gives_identical_results(H, recon, riemann):
    """CTU FP32 in each register-budget variant and several persistent
    grid sizes (the default, a ragged 7, 16 = the XCD-blocked group order
    with an empty last block, one group per workgroup) gives the same bits
    on the box path and the ghosted-groups path."""
    gamma = 1.4
    n = 48
    box = random_smooth_box(n, gamma, 21 + recon + 2 * riemann, amp=0.3)
    B = _dev(W.box_to_groups(box), torch.float32)
    g = H.ghost_width(H.CTU, recon)
    G = H.fill_ghosts_periodic(_dev(box, torch.float32), g)
    spec = H.make_spec(H.CTU, recon, riemann, gamma=gamma, char=True)
    dt = torch.full((1,), 1.5e-3, dtype=torch.float64, device="cuda")
    kw = dict(dh=1 / n, gamma=gamma, scheme=H.CTU, recon=recon, riemann=riemann, char=True)
    outs = []
    try:
        for variant in (4, 2):
            for grid in (0, 7, 16, B.shape[0]):
                H.set_launch_shape(spec, grid, variant)
                ob = torch.empty_like(B)
                H.step_box(B, ob, (n, n, n), dt, **kw)
                og = torch.empty_like(B)
                H.solve_groups(G, og, None, dt=1.5e-3, **kw)
                outs.append(((variant, grid), ob, og))
        torch.cuda.synchronize()
    finally:
        H.set_launch_shape(spec, 0, 4)
    ref_b, ref_g = outs[0][1], outs[0][2]
    assert torch.equal(ref_b, ref_g)
    for shape, ob, og in outs[1:]:
        assert torch.equal(ob, ref_b), shape
        assert torch.equal(og, ref_g), shape


def test_step_box_rejects_plain_and_bad_sizes(H):
    x = torch.zeros((1, 5, 16, 16, 16), device="cuda")
    dt = torch.ones(1, dtype=torch.float64, device="cuda")
    with pytest.raises(H.HydroError):
        H.lib()  # noqa: B018
        rc = H.lib().hydro_step_box(H._ptr(x), H._ptr(x.clone()), None, 24, 16, 16, H._ptr(dt), 1.0, 1.0, 1.4, 2, 1,
                                    1, 1, 0, H._stream())
        H._check("hydro_step_box", rc)
    y = torch.empty_like(x)
    with pytest.raises(H.HydroError):
        H.step_box(x, x, (16, 16, 16), dt, dh=1.0, gamma=1.4, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC)
    ok = torch.zeros_like(x)
    ok[:, 0] = 1.0
    ok[:, 4] = 2.5
    H.step_box(ok, y, (16, 16, 16), dt * 0.01, dh=1.0, gamma=1.4, scheme=H.CTU, recon=H.PPM, riemann=H.HLLC)
    torch.cuda.synchronize()
    assert torch.equal(y, ok)  # a uniform state at rest is a steady state


def test_cfl_dt_batch_equals_single(H):
    gamma = 1.4
    sizes = (32, 48, 16)
    states, rows, first = [], [], 0
    for k, n in enumerate(sizes):
        st = _dev(W.box_to_groups(W.lognormal_blast_box(n, gamma=gamma, seed=30 + k, radius_cells=3)), torch.float32)
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        states.append((st, dt, n))
        rows.append((st, st, None, dt, 1.0, 1.0 / n, first, st.shape[0]))
        first += st.shape[0]
    table = H.seg_table(rows, "cuda")
    H.cfl_dt_batch(table, len(rows), first, gamma=gamma, cfl=0.4)
    for st, dt, n in states:
        single = H.cfl_dt(st, 1.0 / n, gamma, 0.4)
        torch.cuda.synchronize()
        assert dt.item() == single.item()
        assert dt.item() == O.cfl_dt(st.cpu().numpy().astype(np.float64), 1.0 / n, gamma, 0.4)


def _two_state_box(n, left, right, gamma):
    """Box split at x = 1/2 into two uniform primitive states (rho, u, p)."""
    x = (np.arange(n) + 0.5) / n
    sel = (x < 0.5)[None, None, :] * np.ones((n, n, 1), dtype=bool)
    rho = np.where(sel, left[0], right[0])
    u = np.where(sel, left[1], right[1])
    p = np.where(sel, left[2], right[2])
    return W.primitive_to_conserved(rho, u, 0 * u, 0 * u, p, gamma)


@pytest.mark.parametrize("case", ["roe_fallback", "floors"])
def test_diagnostic_counts_do_not_depend_on_launch_shape(H, case):
    """Roe fallbacks (strong double rarefaction) and floor hits (a region
    below the pressure floor) are counted on the device; the totals are the
    same for every launch shape and for the box and ghosted-groups paths,
    in FP32 and FP64."""
    gamma, n = 1.4, 32
    if case == "roe_fallback":
        box = _two_state_box(n, (1.0, -2.0, 0.4), (1.0, 2.0, 0.4), gamma)
        riemann, key = H.ROE, "roe_fallbacks"
    else:
        box = _two_state_box(n, (1.0, 0.0, 1.0), (1e-9, 3.0, 1e-11), gamma)
        riemann, key = H.HLLC, "floor_hits"
    g = H.ghost_width(H.CTU, H.PPM)
    for dtype in (torch.float32, torch.float64):
        B = _dev(W.box_to_groups(box), dtype)
        G = H.fill_ghosts_periodic(_dev(box, dtype), g)
        f64 = dtype == torch.float64
        spec = H.make_spec(H.CTU, H.PPM, riemann, gamma=gamma, char=True, f64=f64)
        dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
        kw = dict(dh=1 / n, gamma=gamma, scheme=H.CTU, recon=H.PPM, riemann=riemann, char=True)
        counts = {}
        try:
            for variant, grid in ((2, 0), (2, 7), (2, 16)) + (() if f64 else ((4, 0), (4, B.shape[0]))):
                H.set_launch_shape(spec, grid, variant)
                H.get_diag(reset=True)
                ob = torch.empty_like(B)
                H.step_box(B, ob, (n, n, n), dt, **kw)
                db = H.get_diag(reset=True)
                og = torch.empty_like(B)
                H.solve_groups(G, og, None, dt=1e-3, **kw)
                dg = H.get_diag(reset=True)
                assert torch.isfinite(ob).all() and torch.equal(ob, og)
                counts[(variant, grid, "box")] = db
                counts[(variant, grid, "groups")] = dg
        finally:
            H.set_launch_shape(spec, 0, 2 if f64 else 4)
        first = next(iter(counts.values()))
        assert first[key] > 0, (dtype, first)
        for shape, d in counts.items():
            assert d == first, (dtype, shape, d, first)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_cfl_dt_sums_bit_identical_to_separate_reductions(H, dtype):
    """The one-pass dt + sums equals hydro_cfl_dt and hydro_conserved_sums
    bit for bit, for group counts that leave ragged slices per workgroup."""
    gamma = 1.4
    rng = np.random.default_rng(44)
    for n in (1, 7, 300, 1031):
        rho = rng.uniform(0.5, 2.0, (n, 4096))
        v = rng.normal(0.0, 0.7, (3, n, 4096))
        p = rng.uniform(0.2, 3.0, (n, 4096))
        U = np.stack([rho, rho * v[0], rho * v[1], rho * v[2],
                      p / (gamma - 1) + 0.5 * rho * (v ** 2).sum(0)], axis=1).reshape(n, 5, 16, 16, 16)
        Ut = _dev(U, dtype)
        dh = 1.0 / 96
        dt1 = H.cfl_dt(Ut, dh, gamma, 0.45)
        s1 = H.conserved_sums(Ut, dh)
        dt2, s2 = H.cfl_dt_sums(Ut, dh, gamma, 0.45)
        torch.cuda.synchronize()
        assert torch.equal(dt1, dt2), (n, dt1.item(), dt2.item())
        assert torch.equal(s1, s2), (n, s1, s2)


def test_vl_box_segments_in_one_launch(H):
    """VL over two periodic boxes of different shapes in one launch: declared
    as boxes (half step once per cell) it equals each box stepped alone bit
    for bit; undeclared (ghosted half step) it agrees to a few ulps; and a
    ghosted-groups segment in a launch declared as boxes comes out NaN while
    the box segment beside it stays finite."""
    gamma = 1.4
    shapes = ((32, 32, 32), (48, 32, 16))
    boxes = [W.lognormal_blast_box(48, gamma=gamma, seed=31 + k, radius_cells=3)[:, :nz, :ny, :nx].copy()
             for k, (nx, ny, nz) in enumerate(shapes)]
    B = [_dev(W.box_to_groups(b), torch.float32) for b in boxes]
    dt_dev = torch.tensor([1.2e-3], dtype=torch.float64, device="cuda")
    kw = dict(gamma=gamma, scheme=H.VL, recon=H.PPM, riemann=H.HLLC, char=True)
    alone = []
    for b, (nx, ny, nz) in zip(B, shapes):
        o = torch.empty_like(b)
        H.step_box(b, o, (nx, ny, nz), dt_dev, dh=1 / 48, **kw)
        alone.append(o)
    n = sum(b.shape[0] for b in B)
    for declared in (True, False):
        outs = [torch.empty_like(b) for b in B]
        rows, first = [], 0
        for b, o, (nx, ny, nz) in zip(B, outs, shapes):
            rows.append((b, o, None, dt_dev, 1.0, 1 / 48, first, b.shape[0], (nx // 16, ny // 16, nz // 16)))
            first += b.shape[0]
        spec = H.make_spec(H.VL, H.PPM, H.HLLC, gamma=gamma, char=True, box_segs=declared)
        H.solve_batch(H.seg_table(rows, "cuda"), len(rows), n, spec)
        torch.cuda.synchronize()
        for o, a in zip(outs, alone):
            if declared:
                assert torch.equal(o, a)
            else:
                assert ((o - a).abs().max() / a.abs().max()).item() <= 4 * 2.0 ** -23
    # A ghosted segment under the box declaration is flagged with NaN.
    g = H.ghost_width(H.VL, H.PPM)
    nx, ny, nz = shapes[0]
    Gh = H.fill_ghosts_periodic(B[0], g, grouped=True, shape=(nx, ny, nz))
    o0, o1 = torch.empty_like(B[0]), torch.empty_like(B[1])
    rows = [(B[1], o1, None, dt_dev, 1.0, 1 / 48, 0, B[1].shape[0], (3, 2, 1)),
            (Gh, o0, None, dt_dev, 1.0, 1 / 48, B[1].shape[0], Gh.shape[0])]
    spec = H.make_spec(H.VL, H.PPM, H.HLLC, gamma=gamma, char=True, box_segs=True)
    H.solve_batch(H.seg_table(rows, "cuda"), len(rows), B[1].shape[0] + Gh.shape[0], spec)
    torch.cuda.synchronize()
    assert torch.isnan(o0).all()
    assert torch.equal(o1, alone[1])


def test_box_segment_beyond_slab_limit_is_nan(H):
    """Box cells are addressed by a 32-bit byte offset within a z-slab of
    groups.  A batched box segment whose slab holds 4 GiB or more (here FP32,
    229 x 229 groups = 52,441 x 80 KiB) gets NaN outputs, for CTU and MHM,
    while a small box segment of the same launch is stepped exactly as alone.
    (hydro_step_box rejects such a box on the host; see tests/test_abi.py.)"""
    gamma, ng = 1.4, 229
    big = torch.zeros((ng * ng, 5, 16, 16, 16), dtype=torch.float32, device="cuda")
    big[:, 0] = 1.0
    big[:, 4] = 1.0 / (gamma - 1.0)
    out_big = torch.empty_like(big)
    small = _dev(W.box_to_groups(W.lognormal_blast_box(32, gamma=gamma, seed=5, radius_cells=3)), torch.float32)
    dt_dev = torch.tensor([1e-4], dtype=torch.float64, device="cuda")
    for scheme in (H.CTU, H.MHM):
        alone = torch.empty_like(small)
        H.step_box(small, alone, (32, 32, 32), dt_dev, dh=1 / 32, gamma=gamma, scheme=scheme, recon=H.PPM,
                   riemann=H.HLLC, char=True)
        out_small = torch.empty_like(small)
        rows = [(small, out_small, None, dt_dev, 1.0, 1 / 32, 0, small.shape[0], (2, 2, 2)),
                (big, out_big, None, dt_dev, 1.0, 1 / 32, small.shape[0], big.shape[0], (ng, ng, 1))]
        spec = H.make_spec(scheme, H.PPM, H.HLLC, gamma=gamma, char=True)
        H.solve_batch(H.seg_table(rows, "cuda"), len(rows), small.shape[0] + big.shape[0], spec)
        torch.cuda.synchronize()
        assert torch.isnan(out_big).all(), scheme
        assert torch.equal(out_small, alone), scheme
    del big, out_big
    torch.cuda.empty_cache()


def test_amr_graph_replay_matches_eager(H):
    """The AMR preparation (group map, padded fill), the flux accumulation and
    the coarse-grid correction captured in a HIP graph: three replays, with
    eager resets of the in-place buffers between them, each equal to the
    eager result bit for bit (no memset node, no allocation inside)."""
    rng = np.random.default_rng(71)
    n, g = 32, 3
    lay = torch.from_numpy(np.array([[0, 16, 16, 16], [0, 32, 16, 16], [0, 48, 16, 16], [0, 0, 48, 0]],
                                    dtype=np.int32)).cuda()
    f32 = torch.float32
    fine = _dev(rng.random((4, 5, 16, 16, 16)) + 1.0, f32)
    c0 = _dev(rng.random((5, 8, 8, 8)) + 1.0, f32)
    c1 = _dev(rng.random((5, 8, 8, 8)) + 1.0, f32)
    coarse0 = _dev(rng.random((8, 5, 16, 16, 16)) + 1.0, f32)
    cflux = _dev(rng.standard_normal((8, 3, 3, 5, 16, 16)), f32)
    fl = _dev(rng.standard_normal((4, 3, 2, 5, 16, 16)), f32)
    amap = torch.empty(H.group_map_len(4, 1), dtype=torch.int32, device="cuda")
    fmap = torch.empty(H.group_map_len(n // 8, 1), dtype=torch.int32, device="cuda")
    pad = torch.empty((4, 5, 22, 22, 22), dtype=f32, device="cuda")
    acc = torch.zeros_like(fl)
    coarse = coarse0.clone()

    def cycle():
        H.build_group_map(lay, 4, 1, out=amap)
        H.build_group_map(lay, n // 8, 1, out=fmap)
        H.fill_groups_amr(fine, lay, amap, 4, [0.25], c0, c1, g, out=pad)
        H.accumulate(acc, fl, 0.5)
        H.amr_correct(coarse, n, cflux, fine, lay, fmap, acc, 1e-3, 1.0 / n)

    def reset():
        acc.zero_()
        coarse.copy_(coarse0)
        pad.zero_()
        amap.zero_()
        fmap.zero_()

    reset()
    cycle()
    torch.cuda.synchronize()
    want = [t.clone() for t in (amap, fmap, pad, acc, coarse)]
    reset()
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        cycle()
    for r in range(3):
        reset()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for got, w in zip((amap, fmap, pad, acc, coarse), want):
            assert torch.equal(got, w), r
    assert not torch.equal(coarse, coarse0)

"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hydro.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hydro_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1103_3373_amd import hydro
    return hydro.lib()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("hydro_solve_groups", "hydro_cfl_dt", "hydro_conserved_sums", "hydro_fill_ghosts_periodic",
              "hydro_solve_batch", "hydro_autotune", "hydro_get_diag", "hydro_last_error", "hydro_shutdown",
              "hydro_ghost_width", "hydro_fill_groups_interp"):
        assert n in names


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_binding_covers_exports():
    from paper_1103_3373_amd import hydro
    assert sorted(hydro.EXPORTS) == _declared()


def test_ghost_widths(L):
    assert [L.hydro_ghost_width(s, r) for s in (0, 1, 2) for r in (0, 1)] == [2, 3, 3, 4, 2, 3]
    assert L.hydro_ghost_width(3, 0) == -1 and L.hydro_ghost_width(0, 2) == -1


def _solve(L, *, inp=0x1000, out=0x100000000, flux=None, n=1, dt=1e-3, dh=1.0, gamma=1.4, scheme=2, recon=1,
           riemann=1, limiter=1, flags=0):
    return L.hydro_solve_groups(ctypes.c_void_p(inp), ctypes.c_void_p(out), ctypes.c_void_p(flux), n, dt, dh, gamma,
                                scheme, recon, riemann, limiter, flags, None)


def test_argument_validation(L):
    EINVAL, EUNSUP, EALIAS = -1, -2, -4
    assert _solve(L, n=0) == 0  # empty batch is a no-op
    assert _solve(L, n=-1) == EINVAL
    assert _solve(L, dt=0.0) == EINVAL
    assert _solve(L, dt=float("nan")) == EINVAL
    assert _solve(L, dh=-1.0) == EINVAL
    assert _solve(L, gamma=1.0) == EINVAL
    assert _solve(L, scheme=3) == EINVAL
    assert _solve(L, recon=2) == EINVAL
    # The exact solver and the Roe -> exact fallback pass validation.  Checked
    # with an empty batch, which returns before any device call, so no kernel
    # is ever launched on the fake addresses even where a GPU is visible.
    assert _solve(L, n=0, riemann=3) == 0
    assert _solve(L, n=0, riemann=0, flags=0x80) == 0
    assert _solve(L, riemann=4) == EINVAL
    # The fused-only box step has no exact solver and no exact fallback.
    P = ctypes.c_void_p
    step = lambda rs, fl: L.hydro_step_box(P(0x1000), P(0x100000000), None, 32, 32, 32, P(0x2000), 1.0, 1.0 / 32,
                                           1.4, 2, 1, rs, 1, fl, None)
    assert step(3, 0) == EUNSUP
    assert step(0, 0x80) == EUNSUP
    # Box cells are addressed by 32-bit byte offsets within a z-slab of
    # groups: a slab of 4 GiB or more is rejected before any device call.
    big = lambda nx, ny, fl: L.hydro_step_box(P(0x1000), P(0x100000000000), None, nx, ny, 16, P(0x2000), 1.0,
                                              1.0 / 32, 1.4, 2, 1, 1, 1, fl, None)
    assert big(16 * 229, 16 * 229, 0) == EINVAL        # 52,441 groups x 80 KiB
    assert b"4 GiB" in L.hydro_last_error()
    assert big(16 * 162, 16 * 162, 0x01) == EINVAL     # FP64: 26,244 groups x 160 KiB
    assert _solve(L, limiter=4) == EINVAL
    assert _solve(L, flags=0x100) == EINVAL
    assert _solve(L, inp=0, out=0x2000) == EINVAL
    # in [0x1000, 0x1000 + 5*22^3*4) overlaps out
    assert _solve(L, inp=0x1000, out=0x1000 + 4096) == EALIAS
    assert _solve(L, inp=0x1000, out=0x100000000, flux=0x100000000 + 64) == EALIAS
    assert L.hydro_last_error()  # message recorded
    assert L.hydro_fill_ghosts_periodic(ctypes.c_void_p(0x1000), 24, 16, 16, 2, 0, ctypes.c_void_p(0x100000000),
                                        None) == EINVAL
    assert L.hydro_cfl_dt(ctypes.c_void_p(0x1000), 0, 1.0, 1.4, 0.5, 0, ctypes.c_void_p(0x2000), None) == EINVAL


def test_product_path_does_not_import_oracle():
    """The HIP binding and package never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_1103_3373_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".hpp", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "oracle/" not in src, f


def test_set_launch_shape_validation():
    """Launch-shape pinning validates its arguments on the host (no device call)."""
    from paper_1103_3373_amd import hydro as H
    ctu = H.make_spec(H.CTU, H.PPM, H.HLLC, gamma=1.4, char=True)
    mhm = H.make_spec(H.MHM, H.PPM, H.HLLC, gamma=1.4, char=True)
    f64 = H.make_spec(H.CTU, H.PPM, H.HLLC, gamma=1.4, char=True, f64=True)
    for bad in ((ctu, 0, 1), (ctu, 0, 3), (ctu, 0, 5), (ctu, -1, 2), (mhm, 0, 3), (f64, 0, 4), (ctu, 0, 4, -1),
                (ctu, 0, 4, 65)):
        with pytest.raises(H.HydroError):
            H.set_launch_shape(*bad)
    H.set_launch_shape(mhm, 0, 4)
    H.set_launch_shape(f64, 512, 2)
    H.set_launch_shape(ctu, 7, 2, 4)
    H.set_launch_shape(ctu, 0, 4)  # back to the default variant and tile depth


def test_cfl_dt_sums_validation(L):
    """Argument checks of the one-pass dt + sums (host only)."""
    EINVAL, EALIAS = -1, -4
    P = ctypes.c_void_p
    assert L.hydro_cfl_dt_sums(P(0x1000), 0, 1.0, 1.4, 0.5, 0, P(0x2000), P(0x3000), None) == EINVAL
    assert L.hydro_cfl_dt_sums(P(0), 4, 1.0, 1.4, 0.5, 0, P(0x2000), P(0x3000), None) == EINVAL
    assert L.hydro_cfl_dt_sums(P(0x1000), 4, 1.0, 1.0, 0.5, 0, P(0x2000), P(0x3000), None) == EINVAL
    assert L.hydro_cfl_dt_sums(P(0x1000), 4, 1.0, 1.4, 0.5, 0x100, P(0x2000), P(0x3000), None) == EINVAL
    assert L.hydro_cfl_dt_sums(P(0x1000), 4, 1.0, 1.4, 0.5, 0, P(0x2000), P(0x2000 - 8), None) == EALIAS


def test_amr_preparation_validation(L):
    """Argument checks of the AMR group map and preparation step (host only)."""
    EINVAL, EALIAS = -1, -4
    P = ctypes.c_void_p
    L.hydro_group_map_len.restype = ctypes.c_longlong
    assert L.hydro_group_map_len(16, 3) == 16 ** 3 + 32 ** 3 + 64 ** 3
    assert L.hydro_group_map_len(0, 1) == -1
    assert L.hydro_group_map_len(2, 0) == -1
    assert L.hydro_group_map_len(2, 9) == -1
    assert L.hydro_group_map_len(1 << 11, 1) == -1  # 2^33 entries
    assert L.hydro_build_group_map(P(0x1000), 4, 0, 1, P(0x2000), None) == EINVAL
    assert L.hydro_build_group_map(P(0x1000), -1, 2, 1, P(0x2000), None) == EINVAL
    assert L.hydro_build_group_map(P(0x1000), 4, 2, 1, P(0), None) == EINVAL
    al = (ctypes.c_double * 2)(0.0, 0.5)
    bad = (ctypes.c_double * 2)(0.0, 1.5)
    fn = L.hydro_fill_groups_amr
    fn.argtypes = [P, P, ctypes.c_int, P, ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                   ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_int, P, P]
    ok = dict(fine=P(0x10000000), lay=P(0x1000), m=P(0x2000), c0=P(0x20000000), c1=P(0x30000000), out=P(0x40000000))

    def call(n=4, ng0=2, nl=2, cn=8, alpha=al, g=3, flags=0, **kw):
        a = dict(ok, **kw)
        return fn(a["fine"], a["lay"], n, a["m"], ng0, nl, a["c0"], a["c1"], cn, alpha, g, flags, a["out"], None)

    assert call(n=-1) == EINVAL
    assert call(ng0=0) == EINVAL
    assert call(g=5) == EINVAL
    assert call(cn=0) == EINVAL
    assert call(alpha=bad) == EINVAL
    assert call(flags=0x02) == EINVAL
    assert call(fine=P(0)) == EINVAL
    assert call(out=P(0x10000000 + 64)) == EALIAS
    assert call(n=0) == 0


def test_amr_correct_validation(L):
    """Argument checks of the coarse-grid correction and accumulate (host only)."""
    EINVAL, EALIAS = -1, -4
    P = ctypes.c_void_p
    c, cf, f, lay, m, ff = P(0x10000000), P(0x20000000), P(0x30000000), P(0x1000), P(0x2000), P(0x40000000)
    fn = L.hydro_amr_correct
    assert fn(c, 24, cf, f, lay, 2, m, ff, 1e-3, 1.0 / 32, 0, None) == EINVAL      # n not a multiple of 16
    assert fn(c, 32, cf, f, lay, -1, m, ff, 1e-3, 1.0 / 32, 0, None) == EINVAL     # n_fine < 0
    assert fn(c, 32, cf, f, lay, 2, m, ff, 0.0, 1.0 / 32, 0, None) == EINVAL       # dt
    assert fn(c, 32, cf, f, lay, 2, m, ff, 1e-3, 1.0 / 32, 0x02, None) == EINVAL   # flags
    assert fn(c, 32, cf, P(0), lay, 2, m, ff, 1e-3, 1.0 / 32, 0, None) == EINVAL   # null
    assert fn(c, 32, P(0x10000000 + 4096), f, lay, 2, m, ff, 1e-3, 1.0 / 32, 0, None) == EALIAS
    assert fn(c, 32, cf, f, lay, 0, m, ff, 1e-3, 1.0 / 32, 0, None) == 0
    acc = L.hydro_accumulate
    assert acc(P(0x1000), P(0x2000), 0.5, -1, 0, None) == EINVAL
    assert acc(P(0x1000), P(0x2000), float("nan"), 4, 0, None) == EINVAL
    assert acc(P(0x1000), P(0x1000 + 4), 0.5, 4, 0, None) == EALIAS
    assert acc(P(0), P(0x2000), 0.5, 4, 0, None) == EINVAL
    assert acc(P(0x1000), P(0x2000), 0.5, 0, 0, None) == 0


def test_noalloc_dt_rejects_sizes_before_device_calls(L):
    """The allocation-free batched dt rejects batches beyond its static
    scratch (and bad arguments) before any device call; an empty batch is a
    no-op.  The fake table address is never dereferenced."""
    from paper_1103_3373_amd import hydro
    P = ctypes.c_void_p
    call = lambda n_segs, n, gamma=1.4, cfl=0.5, flags=0: L.hydro_cfl_dt_batch_noalloc(
        P(0x1000), n_segs, ctypes.c_longlong(n), gamma, cfl, flags, None)
    assert call(1, hydro.NOALLOC_MAX_GROUPS + 1) == -1
    assert b"static scratch" in L.hydro_last_error()
    assert call(1, 1 << 40) == -1
    assert call(-1, 8) == -1
    assert call(1, -8) == -1
    assert call(0, 0) == 0
    assert call(1, 0) == 0


def test_box_launch_shape_defaults_and_pins():
    """Host logic of a box step's launch shape (no device work; the
    compute-unit count is 256 on MI355X and the library's fallback without
    a device): the default tile depth is the largest of 4, 2 that divides
    the box's groups in z and leaves two runs per resident workgroup slot; a
    pinned depth that is not built or does not divide it falls back to the
    largest built divisor below it (depths 2 and 4 exist for the FP32 van
    Leer / characteristic specialization with two workgroups per CU only);
    MHM and VL (second stage) have runs with PPM only."""
    from paper_1103_3373_amd import hydro as H
    ctu = H.make_spec(H.CTU, H.PPM, H.HLLC, gamma=1.4, char=True)
    mhm = H.make_spec(H.MHM, H.PPM, H.HLLC, gamma=1.4, char=True)
    try:
        H.set_launch_shape(ctu, 0, 4, 0)
        assert H.get_launch_shape(ctu, (256, 256, 256)) == (1024, 4, 4)  # 4096 groups: 1024 runs of 4
        assert H.get_launch_shape(ctu, (512, 512, 512)) == (3072, 4, 4)
        assert H.get_launch_shape(ctu, (64, 64, 48))[2] == 1  # 48 groups: too few for runs
        H.set_launch_shape(ctu, 512, 4, 8)
        assert H.get_launch_shape(ctu, (256, 256, 256)) == (512, 4, 4)
        H.set_launch_shape(ctu, 0, 4, 3)
        assert H.get_launch_shape(ctu, (256, 256, 256)) == (2048, 4, 2)
        H.set_launch_shape(ctu, 0, 2, 4)
        assert H.get_launch_shape(ctu, (256, 256, 256)) == (256, 2, 1)
        f64 = H.make_spec(H.CTU, H.PPM, H.HLLC, gamma=1.4, char=True, f64=True)
        H.set_launch_shape(f64, 0, 2, 4)
        assert H.get_launch_shape(f64, (256, 256, 256))[2] == 1
        H.set_launch_shape(f64, 0, 2, 0)
        minmod = H.make_spec(H.CTU, H.PPM, H.HLLC, H.GMINMOD, gamma=1.4, char=True)
        assert H.get_launch_shape(minmod, (256, 256, 256))[2] == 1
        H.set_launch_shape(mhm, 0, 4, 0)
        assert H.get_launch_shape(mhm, (256, 256, 256))[2] == 4  # MHM / VL with PPM have runs too
        vl = H.make_spec(H.VL, H.PPM, H.HLLC, gamma=1.4, char=True)
        assert H.get_launch_shape(vl, (256, 256, 256))[2] == 4
        mhm_plm = H.make_spec(H.MHM, H.PLM, H.HLLC, gamma=1.4, char=True)
        H.set_launch_shape(mhm_plm, 0, 4, 4)
        assert H.get_launch_shape(mhm_plm, (256, 256, 256))[2] == 1  # not built
        with pytest.raises(H.HydroError):
            H.get_launch_shape(ctu, (256, 256, 250))
    finally:
        H.set_launch_shape(ctu, 0, 4, 0)
        H.set_launch_shape(mhm, 0, 4, 0)
        H.set_launch_shape(H.make_spec(H.MHM, H.PLM, H.HLLC, gamma=1.4, char=True), 0, 4, 0)


def test_counter_profile_matches_kernel_sources():
    """The committed rocprofv3 counter summary of the benchmarked CTU kernel
    was taken on the current kernel sources, so bench.py reports the measured
    HBM traffic (roofline.traffic) instead of null; a change to those sources
    needs a new counter run."""
    import importlib.util
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    spec = importlib.util.spec_from_file_location("bench_for_test", os.path.join(root, "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    traffic = bench.traffic_from_profile(bench.kernel_source_hash())
    assert traffic is not None and traffic > 0.671e9  # at least the algorithmic bytes

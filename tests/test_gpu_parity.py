"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.

Bars: FP64 GPU vs oracle <= 1e-12 (scaled max error) after one step and
<= 1e-10 after ten; FP32 GPU vs oracle <= 1e-5 relative L1 and Linf per
conserved variable on smooth data; the FP64 time step is bit-identical
(max is order-free; both sides evaluate the same uncontracted expression);
ghost fills are bit-exact copies.
"""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1103_3373_amd import workloads as W
from tests._util import random_smooth_box, rel_errors, scaled_max_err, var_max_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

COMBOS = list(itertools.product((0, 1, 2), (0, 1), (0, 1, 2), (False, True)))


@pytest.fixture(scope="module")
def H():
    from paper_1103_3373_amd import hydro
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    hydro.lib()
    return hydro


def _dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def _groups(box, scheme, recon):
    g = O.ghost_width(scheme, recon)
    return g, O.fill_ghosts_periodic(box, g)


def _run(H, G, g, dtype, dt, dh, gamma, scheme, recon, rs, lim, char, plain, want_flux=True, flux_mid=False):
    n = G.shape[0]
    inp = _dev(G, dtype)
    out = torch.empty((n, 5, 16, 16, 16), dtype=dtype, device="cuda")
    flux = torch.empty((n, 3, 3 if flux_mid else 2, 5, 16, 16), dtype=dtype, device="cuda") if want_flux else None
    H.solve_groups(inp, out, flux, dt=dt, dh=dh, gamma=gamma, scheme=scheme, recon=recon, riemann=rs, limiter=lim,
                   char=char, plain=plain, flux_mid=flux_mid)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), (flux.cpu().numpy().astype(np.float64) if want_flux else None)


@pytest.mark.parametrize("scheme,recon,rs,char", COMBOS)
@pytest.mark.parametrize("plain", [True, False])
def test_fp64_one_step_matches_oracle(H, scheme, recon, rs, char, plain):
    gamma = 1.4
    box = W.lognormal_blast_box(32, gamma=gamma, seed=7, radius_cells=3)
    g, G = _groups(box, scheme, recon)
    dt, dh = 2e-3, 1 / 32
    flags = (O.F_CHAR if char else 0) | O.F_FLUX_MID
    ref, rflux = O.solve_groups(G, g, dt, dh, gamma, scheme, recon, rs, 1, flags, want_flux=True)
    out, flux = _run(H, G, g, torch.float64, dt, dh, gamma, scheme, recon, rs, 1, char, plain, flux_mid=True)
    assert scaled_max_err(out, ref) <= 1e-12
    assert var_max_err(out, ref) <= 1e-12
    assert scaled_max_err(flux, rflux) <= 1e-12


@pytest.mark.parametrize("lim", [0, 2, 3])
@pytest.mark.parametrize("scheme,recon,char", [(0, 0, False), (1, 1, True), (2, 1, True), (2, 0, False)])
def test_fp64_limiters(H, lim, scheme, recon, char):
    gamma = 5.0 / 3.0
    box = random_smooth_box(32, gamma, 3, amp=0.4)
    g, G = _groups(box, scheme, recon)
    flags = O.F_CHAR if char else 0
    ref, _ = O.solve_groups(G, g, 3e-3, 1 / 32, gamma, scheme, recon, 0, lim, flags)
    for plain in (True, False):
        out, _ = _run(H, G, g, torch.float64, 3e-3, 1 / 32, gamma, scheme, recon, 0, lim, char, plain, False)
        assert scaled_max_err(out, ref) <= 1e-12
        assert var_max_err(out, ref) <= 1e-12


@pytest.mark.parametrize("scheme,recon,rs,char", [(0, 0, 0, False), (1, 1, 1, True), (2, 1, 1, True),
                                                  (2, 0, 2, False)])
def test_fp64_ten_steps_sod_32(H, scheme, recon, rs, char):
    """Sod along x with seeded density noise, 32^3 periodic box as 8 groups,
    gamma 5/3, CFL 0.5, FP64 plain path, 10 steps.

    Every step is first checked from the same input (the oracle's state) at
    1e-12.  The chained 10-step runs are then compared: MHM and VL to 1e-10.
    CTU's characteristic tracing switches a wave's contribution on or off
    with the sign of its speed, and Sod's rest state has u = 0 up to
    round-off, so chained CTU runs that differ only in the last bit take
    different branches there (the oracle alone shows a 1e-15 input
    perturbation growing to ~2e-5 of the field maximum); CTU chains are held
    to 1e-4 of the field maximum."""
    gamma = 5.0 / 3.0
    box = W.sod_box(32, gamma=gamma)
    ref = box.copy()
    g = O.ghost_width(scheme, recon)
    flags = O.F_CHAR if char else 0
    dev = _dev(box, torch.float64)

    def gpu_step(state_dev, dt):
        grp = H.fill_ghosts_periodic(state_dev, g)
        out = torch.empty((8, 5, 16, 16, 16), dtype=torch.float64, device="cuda")
        H.solve_groups(grp, out, None, dt=dt, dh=1 / 32, gamma=gamma, scheme=scheme, recon=recon, riemann=rs,
                       limiter=1, char=char, plain=True)
        return _dev(W.groups_to_box(out.cpu().numpy(), 32, 32, 32), torch.float64)

    for _ in range(10):
        dt = O.cfl_dt(ref, 1 / 32, gamma, 0.5)
        one = gpu_step(_dev(ref, torch.float64), dt).cpu().numpy()
        ref = O.step_box(ref, dt, 1 / 32, gamma, scheme, recon, rs, 1, flags)
        assert scaled_max_err(one, ref) <= 1e-12
        assert var_max_err(one, ref) <= 1e-12
        dev = gpu_step(dev, dt)
    if scheme == 2:
        assert scaled_max_err(dev.cpu().numpy(), ref) <= 1e-4
    else:
        assert scaled_max_err(dev.cpu().numpy(), ref) <= 1e-10


@pytest.mark.parametrize("scheme,recon,rs,char", COMBOS)
def test_fp32_one_step_smooth_within_1e5(H, scheme, recon, rs, char):
    gamma = 1.4
    box = random_smooth_box(32, gamma, 11, amp=0.3)
    g = O.ghost_width(scheme, recon)
    G = O.fill_ghosts_periodic(box, g).astype(np.float32).astype(np.float64)
    dt, dh = 4e-3, 1 / 32
    ref, rflux = O.solve_groups(G, g, dt, dh, gamma, scheme, recon, rs, 1, O.F_CHAR if char else 0,
                                want_flux=True)
    for plain in (True, False):
        out, flux = _run(H, G, g, torch.float32, dt, dh, gamma, scheme, recon, rs, 1, char, plain)
        l1, linf = rel_errors(out, ref)
        assert l1.max() <= 1e-5 and linf.max() <= 1e-5, (l1, linf)
        # Face fluxes: mass / energy fluxes are O(1); compare against the field scale.
        assert scaled_max_err(flux, rflux) <= 1e-5


@pytest.mark.parametrize("lim", [0, 2, 3])
@pytest.mark.parametrize("scheme,recon,rs,char", [(0, 0, 0, False), (0, 1, 1, True), (1, 1, 1, True),
                                                  (1, 0, 2, False), (2, 1, 1, True), (2, 0, 0, False)])
def test_fp32_limiters_smooth_within_1e5(H, lim, scheme, recon, rs, char):
    """Generalized minmod, van Albada and hybrid limiters in FP32 (the
    fused kernels take these through their run-time limiter branch) against
    the oracle on the FP32-rounded input: relative L1 and Linf <= 1e-5 per
    conserved variable, fused and plain paths, with face fluxes."""
    gamma = 1.4
    box = random_smooth_box(32, gamma, 17 + lim, amp=0.3)
    g = O.ghost_width(scheme, recon)
    G = O.fill_ghosts_periodic(box, g).astype(np.float32).astype(np.float64)
    dt, dh = 4e-3, 1 / 32
    ref, rflux = O.solve_groups(G, g, dt, dh, gamma, scheme, recon, rs, lim, O.F_CHAR if char else 0,
                                want_flux=True)
    for plain in (True, False):
        out, flux = _run(H, G, g, torch.float32, dt, dh, gamma, scheme, recon, rs, lim, char, plain)
        l1, linf = rel_errors(out, ref)
        assert l1.max() <= 1e-5 and linf.max() <= 1e-5, (plain, l1, linf)
        fl1, flinf = rel_errors(flux, rflux, axis=3)  # [n][dir][face][var][16][16]
        assert flinf.max() <= 1e-5, (plain, fl1, flinf)


@pytest.mark.parametrize("scheme,recon,rs", [(0, 1, 0), (1, 1, 1), (2, 1, 1), (2, 1, 0)])
def test_fp32_blast_shocks(H, scheme, recon, rs):
    """Lognormal + blasts with shocks: FP32 stays within 1e-5 in relative L1."""
    gamma = 1.4
    box = W.lognormal_blast_box(32, gamma=gamma, seed=9, radius_cells=4)
    g = O.ghost_width(scheme, recon)
    G = O.fill_ghosts_periodic(box, g).astype(np.float32).astype(np.float64)
    dt = O.cfl_dt(box, 1 / 32, gamma, 0.5 if scheme == 2 else 0.3)
    ref, _ = O.solve_groups(G, g, dt, 1 / 32, gamma, scheme, recon, rs, 1, O.F_CHAR)
    out, _ = _run(H, G, g, torch.float32, dt, 1 / 32, gamma, scheme, recon, rs, 1, True, False, False)
    l1, linf = rel_errors(out, ref)
    assert l1.max() <= 1e-5, (l1, linf)


def test_ragged_batches_and_empty(H):
    """Group counts that do not fill the launch (1, 3, 7, 9) and n = 0."""
    gamma = 1.4
    box = random_smooth_box(48, gamma, 5, amp=0.3, nz=48)
    for scheme, recon in ((2, 1), (0, 0), (1, 1)):
        g, G = _groups(box, scheme, recon)
        ref, _ = O.solve_groups(G[:9], g, 3e-3, 1 / 48, gamma, scheme, recon, 1, 1, O.F_CHAR)
        for n in (1, 3, 7, 9):
            for plain in (True, False):
                out, _ = _run(H, G[:n], g, torch.float64, 3e-3, 1 / 48, gamma, scheme, recon, 1, 1, True, plain,
                              False)
                assert scaled_max_err(out, ref[:n]) <= 1e-12
                assert var_max_err(out, ref[:n]) <= 1e-12
    z = torch.empty((0, 5, 22, 22, 22), dtype=torch.float32, device="cuda")
    H.solve_groups(z, torch.empty((0, 5, 16, 16, 16), device="cuda"), None, dt=1e-3, dh=1.0, gamma=1.4, scheme=2,
                   recon=1, riemann=1)


def test_free_stream_bitwise(H):
    gamma = 1.4
    one = np.ones((32, 32, 32))
    box = W.primitive_to_conserved(1.3 * one, 0.2 * one, -0.4 * one, 0.1 * one, 0.9 * one, gamma)
    for scheme, recon in ((0, 0), (1, 1), (2, 1)):
        g, G = _groups(box, scheme, recon)
        for dtype in (torch.float32, torch.float64):
            for plain in (True, False):
                out, _ = _run(H, G, g, dtype, 1e-2, 1 / 32, gamma, scheme, recon, 0, 1, True, plain, False)
                want = W.box_to_groups(box).astype(np.float32 if dtype == torch.float32 else np.float64)
                np.testing.assert_array_equal(out, want.astype(np.float64))


def test_roe_fallback_counted(H):
    """Strong double rarefaction trips the Roe positivity test (paper Sec. 2)."""
    gamma = 1.4
    x = (np.arange(32) + 0.5) / 32
    u = np.where(x < 0.5, -2.0, 2.0)[None, None, :] * np.ones((32, 32, 1))
    box = W.primitive_to_conserved(np.ones_like(u), u, 0 * u, 0 * u, 0.4 * np.ones_like(u), gamma)
    g, G = _groups(box, 2, 0)
    O.reset_stats()
    ref, _ = O.solve_groups(G, g, 2e-3, 1 / 32, gamma, 2, 0, 0, 1, 0)
    n_ref = O.stats()["roe_fail"]
    assert n_ref > 0
    for plain in (True, False):
        H.get_diag(reset=True)
        out, _ = _run(H, G, g, torch.float64, 2e-3, 1 / 32, gamma, 2, 0, 0, 1, False, plain, False)
        d = H.get_diag(reset=True)
        assert scaled_max_err(out, ref) <= 1e-12
        assert var_max_err(out, ref) <= 1e-12
        assert d["roe_fallbacks"] >= 1


def test_dt_bit_exact_on_upcast_fp32_state(H):
    gamma = 1.4
    box = W.lognormal_blast_box(64, gamma=gamma, seed=2)
    grp32 = W.box_to_groups(box).astype(np.float32)
    want = O.cfl_dt(grp32.astype(np.float64), 1 / 64, gamma, 0.5)
    got = H.cfl_dt(_dev(grp32, torch.float32), 1 / 64, gamma, 0.5).item()
    assert got == want
    got64 = H.cfl_dt(_dev(W.box_to_groups(box), torch.float64), 1 / 64, gamma, 0.5).item()
    assert got64 == O.cfl_dt(W.box_to_groups(box), 1 / 64, gamma, 0.5)


def test_conserved_sums(H):
    box = W.lognormal_blast_box(64, gamma=1.4, seed=3)
    grp = W.box_to_groups(box)
    want = O.conserved_sums(grp, 1 / 64)
    for dtype in (torch.float64, torch.float32):
        src = grp if dtype == torch.float64 else grp.astype(np.float32).astype(np.float64)
        ref = O.conserved_sums(src, 1 / 64)
        a = H.conserved_sums(_dev(src, dtype), 1 / 64).cpu().numpy()
        b = H.conserved_sums(_dev(src, dtype), 1 / 64).cpu().numpy()
        np.testing.assert_array_equal(a, b)  # deterministic
        scale = O.conserved_sums(np.abs(src), 1 / 64)
        assert np.all(np.abs(a - ref) <= 1e-13 * scale)
    assert want.shape == (5,)


@pytest.mark.parametrize("g", [2, 3, 4, 5])
def test_periodic_ghost_fill_bit_exact(H, g):
    rng = np.random.default_rng(g)
    box = rng.standard_normal((5, 32, 48, 16))
    want = O.fill_ghosts_periodic(box, g)
    got = H.fill_ghosts_periodic(_dev(box, torch.float64), g).cpu().numpy()
    np.testing.assert_array_equal(got, want)
    grouped = _dev(W.box_to_groups(box), torch.float64)
    got2 = H.fill_ghosts_periodic(grouped, g, grouped=True, shape=(16, 48, 32)).cpu().numpy()
    np.testing.assert_array_equal(got2, want)


@pytest.mark.parametrize("g", [2, 3, 4, 5])
@pytest.mark.parametrize("cn", [16, 64])
def test_interp_fill_matches_oracle(H, g, cn):
    """Trilinear preparation of AMR-shaped groups against the oracle (which
    sums the eight weighted corners; the kernels interpolate axis by axis,
    so the FP64 results agree to rounding).  g = 5 takes the generic
    kernel.  Levels of 32, 64 and 128 cells per side: the 16^3 coarse field
    is coarser than all of them (coarse layers shared by fine planes); the
    64^3 one is finer than level 0 (layers skipped), as fine as level 1 (a
    new layer every plane) and coarser than level 2."""
    coarse = W.amr_coarse_field(cn, seed=5)
    lay = W.amr_layout((3, 5, 7), base_n=32, seed=5)
    want = O.fill_groups_interp(coarse, lay, g, 1 / 32)
    got = H.fill_groups_interp(_dev(coarse, torch.float64), torch.from_numpy(lay).cuda(), g, 1 / 32).cpu().numpy()
    assert scaled_max_err(got, want) <= 1e-15
    got32 = H.fill_groups_interp(_dev(coarse, torch.float32), torch.from_numpy(lay).cuda(), g, 1 / 32).cpu().numpy()
    assert scaled_max_err(got32, want) <= 2e-7


def test_full_size_sampled_groups(H):
    """256^3 (4096 groups), FP32 CTU+PPM(char)+HLLC as benchmarked: sampled
    groups against the oracle, every output finite, conservation of the
    whole box to FP32 round-off."""
    gamma = 1.4
    box = W.lognormal_blast_box(256, gamma=gamma, seed=W.IC_SEED)
    g = 3
    dev_box = _dev(box, torch.float32)
    grp = H.fill_ghosts_periodic(dev_box, g)
    dt = O.cfl_dt(box.astype(np.float32).astype(np.float64), 1 / 256, gamma, 0.5)
    out = torch.empty((4096, 5, 16, 16, 16), dtype=torch.float32, device="cuda")
    H.solve_groups(grp, out, None, dt=dt, dh=1 / 256, gamma=gamma, scheme=2, recon=1, riemann=1, limiter=1, char=True)
    torch.cuda.synchronize()
    assert torch.isfinite(out).all().item()
    pick = [0, 1, 777, 2048, 4095]
    G = grp[pick].cpu().numpy().astype(np.float64)
    ref, _ = O.solve_groups(G, g, dt, 1 / 256, gamma, 2, 1, 1, 1, O.F_CHAR)
    l1, linf = rel_errors(out[pick].cpu().numpy(), ref)
    assert l1.max() <= 1e-5, (l1, linf)
    s0 = H.conserved_sums(_dev(W.box_to_groups(box).astype(np.float32), torch.float32), 1 / 256).cpu().numpy()
    s1 = H.conserved_sums(out, 1 / 256).cpu().numpy()
    assert abs(s1[0] - s0[0]) <= 1e-6 * s0[0] and abs(s1[4] - s0[4]) <= 1e-6 * s0[4]


def _amr_case(ng0, counts, cn, seed):
    rng = np.random.default_rng(seed)
    lay = W.amr_layout(counts, base_n=16 * ng0, seed=seed)
    n = lay.shape[0]
    fine = W.amr_coarse_field(16, seed=seed)[None].repeat(n, 0) * (1 + 0.1 * rng.random((n, 1, 1, 1, 1)))
    fine = np.ascontiguousarray(fine)
    c0 = W.amr_coarse_field(cn, seed=seed + 1)
    c1 = c0 * (1 + 0.05 * rng.standard_normal(c0.shape))
    return lay, fine, c0, c1


def test_group_map_matches_numpy(H):
    """Per-level group map: -1 where no group, the group index elsewhere;
    duplicate positions keep the higher index; an origin off the 16-cell grid
    is left out."""
    ng0, n_levels = 2, 3
    lay = W.amr_layout((5, 20, 60), base_n=32, seed=21)
    lay = np.concatenate([lay, lay[3:4], np.array([[1, 8, 0, 0]], dtype=np.int32)]).astype(np.int32)
    want = np.full(H.group_map_len(ng0, n_levels), -1, dtype=np.int32)
    off = 0
    offs = []
    for lv in range(n_levels):
        offs.append(off)
        off += (ng0 << lv) ** 3
    for G, (lv, ox, oy, oz) in enumerate(lay):
        if ox % 16 or oy % 16 or oz % 16:
            continue
        ng = ng0 << lv
        q = offs[lv] + ((oz // 16) * ng + oy // 16) * ng + ox // 16
        want[q] = max(want[q], G)
    got = H.build_group_map(torch.from_numpy(lay).cuda(), ng0, n_levels).cpu().numpy()
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("g", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("cn", [8, 64])
def test_amr_fill_matches_oracle(H, g, dtype, cn):
    """Preparation with same-level neighbours and time-blended coarse ghosts
    on three sparse levels: copied cells bit for bit, interpolated cells to
    FP64 rounding (the oracle sums eight weighted corners, the kernel
    interpolates axis by axis) or to FP32 rounding of the result.  With the
    8^3 coarse field every group's coarse footprint is staged in LDS; the
    64^3 one is too fine for that, so every column reads it directly."""
    ng0, alpha = 2, [0.0, 0.25, 0.625]
    lay, fine, c0, c1 = _amr_case(ng0, (4, 12, 40), cn, 31)
    if dtype == torch.float32:
        fine, c0, c1 = (a.astype(np.float32).astype(np.float64) for a in (fine, c0, c1))
    want = O.fill_groups_amr(fine, lay, ng0, alpha, c0, c1, g)
    lay_d = torch.from_numpy(lay).cuda()
    gmap = H.build_group_map(lay_d, ng0, len(alpha))
    got = H.fill_groups_amr(_dev(fine, dtype), lay_d, gmap, ng0, alpha, _dev(c0, dtype), _dev(c1, dtype), g)
    got = got.cpu().numpy().astype(np.float64)
    if dtype == torch.float64:
        assert scaled_max_err(got, want) <= 1e-15
    else:
        assert scaled_max_err(got, want) <= 2e-7
    # Interiors and neighbour copies are exact copies of the fine values.
    N = 16 + 2 * g
    inner = np.zeros((N, N, N), dtype=bool)
    inner[g:g + 16, g:g + 16, g:g + 16] = True
    np.testing.assert_array_equal(got[:, :, inner], want[:, :, inner])
    nl = [16 * (ng0 << lv) for lv in range(3)]
    cover = {lv: np.zeros((nl[lv],) * 3, dtype=bool) for lv in range(3)}
    for lv, ox, oy, oz in lay:
        cover[lv][oz:oz + 16, oy:oy + 16, ox:ox + 16] = True
    for G, (lv, ox, oy, oz) in enumerate(lay):
        idx = [(np.arange(N) - g + o) % nl[lv] for o in (ox, oy, oz)]
        m = cover[lv][np.ix_(idx[2], idx[1], idx[0])]
        np.testing.assert_array_equal(got[G][:, m], want[G][:, m])


def test_amr_fill_full_level_is_periodic_fill(H):
    """A fully covered level: the preparation equals the periodic ghost fill
    of the level's box bit for bit (no coarse value is used)."""
    rng = np.random.default_rng(41)
    lay = np.array([[0, 16 * x, 16 * y, 16 * z] for z in range(2) for y in range(2) for x in range(2)],
                   dtype=np.int32)
    fine = rng.standard_normal((8, 5, 16, 16, 16))
    box = W.groups_to_box(fine, 32, 32, 32)
    lay_d = torch.from_numpy(lay).cuda()
    gmap = H.build_group_map(lay_d, 2, 1)
    c = _dev(np.full((5, 4, 4, 4), 7.0), torch.float64)
    got = H.fill_groups_amr(_dev(fine, torch.float64), lay_d, gmap, 2, [0.5], c, c, 3).cpu().numpy()
    want = H.fill_ghosts_periodic(_dev(box, torch.float64), 3).cpu().numpy()
    np.testing.assert_array_equal(got, want)


def _fine_layout_32():
    # Fine-grid origins (64^3 fine grid over a 32^3 coarse box): two adjacent
    # groups, one across the periodic boundary from them, one isolated.
    return np.array([[0, 16, 16, 16], [0, 32, 16, 16], [0, 48, 16, 16], [0, 0, 48, 0]], dtype=np.int32)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_amr_correct_matches_oracle(H, dtype):
    """Refluxing and restriction on random data against the oracle: FP64 bit
    for bit (same expressions in the same order), FP32 to its rounding."""
    rng = np.random.default_rng(51)
    n = 32
    lay = _fine_layout_32()
    coarse = rng.standard_normal((8, 5, 16, 16, 16)) + 3.0
    cflux = rng.standard_normal((8, 3, 3, 5, 16, 16))
    fine = rng.standard_normal((4, 5, 16, 16, 16)) + 3.0
    fflux = rng.standard_normal((4, 3, 2, 5, 16, 16))
    if dtype == torch.float32:
        coarse, cflux, fine, fflux = (a.astype(np.float32).astype(np.float64) for a in (coarse, cflux, fine, fflux))
    dt, dh = 2e-3, 1.0 / n
    want = O.amr_correct(coarse, (n, n, n), cflux, fine, lay, fflux, dt, dh)
    lay_d = torch.from_numpy(lay).cuda()
    fmap = H.build_group_map(lay_d, n // 8, 1)
    got = _dev(coarse, dtype)
    H.amr_correct(got, n, _dev(cflux, dtype), _dev(fine, dtype), lay_d, fmap, _dev(fflux, dtype), dt, dh)
    got = got.cpu().numpy().astype(np.float64)
    if dtype == torch.float64:
        np.testing.assert_array_equal(got, want)
    else:
        assert scaled_max_err(got, want) <= 2e-7
    assert not np.array_equal(want, coarse)


def test_amr_cycle_conserves_on_gpu(H):
    """A whole two-level step on the GPU in FP64: the coarse step (fluxes on
    every patch face), two fine sub-steps prepared by the AMR fill at the
    sub-step times, the flux average, then the coarse-grid correction.  The
    domain totals are conserved to round-off and the result matches the
    same cycle run by the oracle."""
    gamma = 1.4
    n = 32
    dh = 1.0 / n
    box = W.lognormal_blast_box(n, gamma=gamma, seed=17, radius_cells=3)
    lay = _fine_layout_32()
    fine0 = np.stack([np.repeat(np.repeat(np.repeat(
        box[:, o[3] // 2:o[3] // 2 + 8, o[2] // 2:o[2] // 2 + 8, o[1] // 2:o[1] // 2 + 8], 2, 1), 2, 2), 2, 3)
        for o in lay])
    g = 3
    dt = O.cfl_dt(box, dh, gamma, 0.4)
    # Oracle cycle.
    cg, cflux = O.solve_groups(O.fill_ghosts_periodic(box, g), g, dt, dh, gamma, 2, 1, 1, 1,
                               O.F_CHAR | O.F_FLUX_MID, want_flux=True)
    new_box = W.groups_to_box(cg, n, n, n)
    fine, fflux = fine0, np.zeros((4, 3, 2, 5, 16, 16))
    for s in range(2):
        pad = O.fill_groups_amr(fine, lay, 4, [0.5 * s], box, new_box, g)
        fine, fl = O.solve_groups(pad, g, 0.5 * dt, 0.5 * dh, gamma, 2, 1, 1, 1, O.F_CHAR, want_flux=True)
        fflux += 0.5 * fl
    want = O.amr_correct(cg, (n, n, n), cflux, fine, lay, fflux, dt, dh)
    # GPU cycle.
    f64 = torch.float64
    c_old = _dev(box, f64)
    grp = H.fill_ghosts_periodic(c_old, g)
    c_new = torch.empty((8, 5, 16, 16, 16), dtype=f64, device="cuda")
    c_flux = torch.empty((8, 3, 3, 5, 16, 16), dtype=f64, device="cuda")
    H.solve_groups(grp, c_new, c_flux, dt=dt, dh=dh, gamma=gamma, scheme=2, recon=1, riemann=1, char=True,
                   flux_mid=True)
    c_new_box = torch.from_numpy(W.groups_to_box(c_new.cpu().numpy(), n, n, n)).cuda()
    lay_d = torch.from_numpy(lay).cuda()
    fmap = H.build_group_map(lay_d, n // 8, 1)
    amap = H.build_group_map(lay_d, 4, 1)
    f_state = _dev(fine0, f64)
    f_acc = torch.zeros((4, 3, 2, 5, 16, 16), dtype=f64, device="cuda")
    f_flux = torch.empty_like(f_acc)
    for s in range(2):
        pad = H.fill_groups_amr(f_state, lay_d, amap, 4, [0.5 * s], c_old, c_new_box, g)
        f_next = torch.empty_like(f_state)
        H.solve_groups(pad, f_next, f_flux, dt=0.5 * dt, dh=0.5 * dh, gamma=gamma, scheme=2, recon=1, riemann=1,
                       char=True)
        H.accumulate(f_acc, f_flux, 0.5)
        f_state = f_next
    H.amr_correct(c_new, n, c_flux, f_state, lay_d, fmap, f_acc, dt, dh)
    got = c_new.cpu().numpy()
    assert scaled_max_err(got, want) <= 1e-12
    t0 = box.reshape(5, -1).sum(1)
    t1 = W.groups_to_box(got, n, n, n).reshape(5, -1).sum(1)
    assert np.abs(t1 - t0).max() <= 1e-13 * np.abs(t0).max()


@pytest.mark.parametrize("scheme,recon,char", [(0, 0, False), (0, 1, True), (1, 0, True), (1, 1, False),
                                               (2, 0, False), (2, 1, True)])
def test_fp64_exact_solver_matches_oracle(H, scheme, recon, char):
    """The exact Riemann solver (plain path) on a blast field with shocks and
    rarefactions against the oracle's exact solver: Newton to a relative
    change below 1e-15 on both sides, so the FP64 results agree to 1e-12."""
    gamma = 1.4
    box = W.lognormal_blast_box(32, gamma=gamma, seed=23, radius_cells=3)
    g, G = _groups(box, scheme, recon)
    G = G[:3]
    dt = O.cfl_dt(box, 1 / 32, gamma, 0.5 if scheme == 2 else 0.3)
    flags = (O.F_CHAR if char else 0) | O.F_FLUX_MID
    ref, rflux = O.solve_groups(G, g, dt, 1 / 32, gamma, scheme, recon, 3, 1, flags, want_flux=True)
    out, flux = _run(H, G, g, torch.float64, dt, 1 / 32, gamma, scheme, recon, 3, 1, char, False, flux_mid=True)
    assert scaled_max_err(out, ref) <= 1e-12
    assert var_max_err(out, ref) <= 1e-12
    assert scaled_max_err(flux, rflux) <= 1e-12


def test_fp32_exact_solver_smooth(H):
    """FP32 exact solver (Newton to 1e-6) within 1e-5 of the FP64 oracle."""
    gamma = 1.4
    box = random_smooth_box(32, gamma, 11, amp=0.3)
    for scheme, recon in ((2, 1), (0, 0)):
        g = O.ghost_width(scheme, recon)
        G = O.fill_ghosts_periodic(box, g).astype(np.float32).astype(np.float64)[:2]
        ref, _ = O.solve_groups(G, g, 4e-3, 1 / 32, gamma, scheme, recon, 3, 1, O.F_CHAR)
        out, _ = _run(H, G, g, torch.float32, 4e-3, 1 / 32, gamma, scheme, recon, 3, 1, True, False, False)
        l1, linf = rel_errors(out, ref)
        assert l1.max() <= 1e-5 and linf.max() <= 1e-5, (l1, linf)


def test_roe_exact_fallback(H):
    """Strong double rarefaction: with the exact fallback every face where
    the Roe linearization fails takes the exact flux (plain path), matching
    the oracle with the same fallback; the failures are still counted."""
    gamma = 1.4
    x = (np.arange(32) + 0.5) / 32
    u = np.where(x < 0.5, -2.0, 2.0)[None, None, :] * np.ones((32, 32, 1))
    box = W.primitive_to_conserved(np.ones_like(u), u, 0 * u, 0 * u, 0.4 * np.ones_like(u), gamma)
    g, G = _groups(box, 2, 0)
    ref_exact, _ = O.solve_groups(G, g, 2e-3, 1 / 32, gamma, 2, 0, 0, 1, O.F_ROE_FB_EXACT)
    ref_hlle, _ = O.solve_groups(G, g, 2e-3, 1 / 32, gamma, 2, 0, 0, 1, 0)
    assert scaled_max_err(ref_exact, ref_hlle) > 1e-8  # the fallback flux matters here
    inp = _dev(G, torch.float64)
    out = torch.empty((G.shape[0], 5, 16, 16, 16), dtype=torch.float64, device="cuda")
    H.get_diag(reset=True)
    H.solve_groups(inp, out, None, dt=2e-3, dh=1 / 32, gamma=gamma, scheme=2, recon=0, riemann=0, limiter=1,
                   roe_fb_exact=True)
    d = H.get_diag(reset=True)
    assert scaled_max_err(out.cpu().numpy(), ref_exact) <= 1e-12
    assert d["roe_fallbacks"] >= 1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_accumulate(H, dtype):
    """acc += w x evaluated in FP64 and rounded to the buffer type, also with
    acc and x the same buffer; the sub-step average of two flux arrays."""
    rng = np.random.default_rng(61)
    a = rng.standard_normal(1000)
    x = rng.standard_normal(1000)
    if dtype == torch.float32:
        a, x = a.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64)
    acc = _dev(a, dtype)
    H.accumulate(acc, _dev(x, dtype), 0.375)
    want = a + 0.375 * x
    got = acc.cpu().numpy().astype(np.float64)
    if dtype == torch.float64:
        np.testing.assert_array_equal(got, want)
    else:
        np.testing.assert_array_equal(got, want.astype(np.float32).astype(np.float64))
    H.accumulate(acc, acc, -0.5)
    np.testing.assert_allclose(acc.cpu().numpy().astype(np.float64), 0.5 * got, rtol=1e-7 if dtype == torch.float32 else 0)

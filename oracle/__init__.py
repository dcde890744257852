"""FP64 CPU oracle of the directionally unsplit hydro schemes (arXiv:1103.3373, Sec. 2).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, plain reference that the
HIP library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: the numerics live in ``oracle.cpp``,
this module only compiles it and marshals numpy arrays through ctypes.

Every array is float64 and C-contiguous.  Layouts follow the paper's flattened
``[var][z][y][x]`` order (Sec. 3.1), variables (rho, mx, my, mz, E).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
LIB = os.path.join(_HERE, "liboracle.so")
LIB_COUNT = os.path.join(_HERE, "liboracle_count.so")

MHM, VL, CTU = 0, 1, 2
PLM, PPM = 0, 1
ROE, HLLC, HLLE, EXACT = 0, 1, 2, 3
GMINMOD, VANLEER, VANALBADA, HYBRID = 0, 1, 2, 3
F_CHAR, F_FLUX_MID, F_ROE_FB_HLLC, F_ROE_FB_EXACT = 0x02, 0x04, 0x10, 0x80
# Oracle-only switches (the HIP library has neither): the unlimited centred
# slope, and no PPM edge clipping or monotonization.  They let the pins check
# the convergence of the linear scheme underneath the limiters.
CENTRAL = 4
F_NO_MONO = 0x100


def build(force: bool = True) -> None:
    """Compile the oracle (plain and op-counting builds) with g++."""
    flags = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-std=c++17"]
    for out, extra in ((LIB, []), (LIB_COUNT, ["-DORACLE_COUNT_OPS"])):
        if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
            tmp = out + ".tmp"
            subprocess.check_call(["g++", *flags, *extra, _SRC, "-o", tmp])
            os.replace(tmp, out)


_libs: dict[str, ctypes.CDLL] = {}


def _lib(counting: bool = False) -> ctypes.CDLL:
    path = LIB_COUNT if counting else LIB
    if path in _libs:
        return _libs[path]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build(force=False)
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i, d = ctypes.c_int, ctypes.c_double
    L.oracle_step_box.argtypes = [P, P, i, i, i, d, d, d, i, i, i, i, i]
    L.oracle_step_box.restype = i
    L.oracle_solve_groups.argtypes = [P, P, P, i, i, d, d, d, i, i, i, i, i]
    L.oracle_solve_groups.restype = i
    L.oracle_fill_ghosts_periodic.argtypes = [P, i, i, i, i, P]
    L.oracle_fill_ghosts_periodic.restype = i
    L.oracle_fill_groups_interp.argtypes = [P, i, P, i, i, d, P]
    L.oracle_fill_groups_interp.restype = i
    L.oracle_fill_groups_amr.argtypes = [P, P, i, i, i, P, P, i, P, i, P]
    L.oracle_fill_groups_amr.restype = i
    L.oracle_amr_correct.argtypes = [P, i, i, i, P, P, P, i, P, d, d]
    L.oracle_amr_correct.restype = i
    L.oracle_cfl_dt.argtypes = [P, ctypes.c_long, ctypes.c_long, d, d, d]
    L.oracle_cfl_dt.restype = d
    L.oracle_conserved_sums.argtypes = [P, ctypes.c_long, ctypes.c_long, d, P]
    L.oracle_conserved_sums.restype = None
    L.oracle_riemann_flux.argtypes = [P, P, i, d, i, i, P]
    L.oracle_riemann_flux.restype = i
    L.oracle_roe_ok.argtypes = [P, P, d]
    L.oracle_roe_ok.restype = i
    L.oracle_exact_riemann.argtypes = [P, P, d, P, P, i, P]
    L.oracle_exact_riemann.restype = i
    L.oracle_limiter.argtypes = [d, d, i]
    L.oracle_limiter.restype = d
    L.oracle_slope.argtypes = [P, P, P, i, d, i, i, P]
    L.oracle_slope.restype = None
    L.oracle_ppm_edge.argtypes = [P, P, P, P, P]
    L.oracle_ppm_edge.restype = None
    L.oracle_char.argtypes = [P, P, d, P, P]
    L.oracle_char.restype = None
    L.oracle_ctu_trace.argtypes = [P, P, P, i, d, d, P, P]
    L.oracle_ctu_trace.restype = None
    L.oracle_ppm_monotonize.argtypes = [P, P, P]
    L.oracle_ppm_monotonize.restype = None
    L.oracle_ghost_width.argtypes = [i, i]
    L.oracle_ghost_width.restype = i
    L.oracle_get_stats.argtypes = [P]
    L.oracle_get_stats.restype = None
    L.oracle_reset_stats.argtypes = []
    L.oracle_reset_stats.restype = None
    L.oracle_get_ops.argtypes = []
    L.oracle_get_ops.restype = ctypes.c_ulonglong
    L.oracle_reset_ops.argtypes = []
    L.oracle_reset_ops.restype = None
    _libs[path] = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def ghost_width(scheme: int, recon: int) -> int:
    """Minimum ghost width of the scheme / reconstruction stencil."""
    return _lib().oracle_ghost_width(scheme, recon)


def step_box(U, dt, dh, gamma, scheme, recon, riemann, limiter, flags=0, counting=False) -> np.ndarray:
    """One step on a periodic box U[5][nz][ny][nx]."""
    U = _f64(U)
    assert U.ndim == 4 and U.shape[0] == 5
    out = np.empty_like(U)
    nz, ny, nx = U.shape[1:]
    rc = _lib(counting).oracle_step_box(_p(U), _p(out), nx, ny, nz, dt, dh, gamma, scheme, recon, riemann,
                                        limiter, flags)
    if rc != 0:
        raise ValueError(f"oracle_step_box failed ({rc})")
    return out


def solve_groups(G, g, dt, dh, gamma, scheme, recon, riemann, limiter, flags=0, want_flux=False,
                 counting=False):
    """One step on padded groups G[n][5][N][N][N] -> (out[n][5][16][16][16], flux or None)."""
    G = _f64(G)
    n = G.shape[0]
    N = 16 + 2 * g
    assert G.shape == (n, 5, N, N, N), G.shape
    out = np.empty((n, 5, 16, 16, 16))
    nf = 3 if flags & F_FLUX_MID else 2
    flux = np.empty((n, 3, nf, 5, 16, 16)) if want_flux else None
    rc = _lib(counting).oracle_solve_groups(_p(G), _p(out), _p(flux) if want_flux else None, n, g, dt, dh,
                                            gamma, scheme, recon, riemann, limiter, flags)
    if rc != 0:
        raise ValueError(f"oracle_solve_groups failed ({rc})")
    return out, flux


def _solve_chunk(args):
    return solve_groups(*args)[0]


class GroupPool:
    """Worker processes that each run solve_groups on a share of a batch of
    patch groups: the host-side analog of threading one step over patches
    (Sec. 4.3).  The arithmetic of every group is solve_groups's own; only
    the groups are split between processes (spawned, so a parent that has
    initialised a GPU is never forked)."""

    def __init__(self, workers: int):
        import multiprocessing as mp
        self.workers = int(workers)
        self._pool = mp.get_context("spawn").Pool(self.workers, initializer=_lib)

    def solve_groups(self, G, g, dt, dh, gamma, scheme, recon, riemann, limiter, flags=0) -> np.ndarray:
        """out[n][5][16][16][16] of solve_groups(G, ...), groups split in
        contiguous chunks (a few per worker)."""
        G = _f64(G)
        chunks = [c for c in np.array_split(np.arange(G.shape[0]), 4 * self.workers) if len(c)]
        outs = self._pool.map(_solve_chunk, [(G[c[0]:c[-1] + 1], g, dt, dh, gamma, scheme, recon, riemann,
                                              limiter, flags) for c in chunks])
        return np.concatenate(outs) if outs else np.empty((0, 5, 16, 16, 16))

    def close(self):
        self._pool.close()
        self._pool.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def fill_ghosts_periodic(box, g) -> np.ndarray:
    """box[5][nz][ny][nx] -> padded groups [G][5][16+2g]^3 (periodic wrap)."""
    box = _f64(box)
    nz, ny, nx = box.shape[1:]
    N = 16 + 2 * g
    n = (nx // 16) * (ny // 16) * (nz // 16)
    out = np.empty((n, 5, N, N, N))
    rc = _lib().oracle_fill_ghosts_periodic(_p(box), nx, ny, nz, g, _p(out))
    if rc != 0:
        raise ValueError("oracle_fill_ghosts_periodic failed")
    return out


def fill_groups_interp(coarse, layout, g, base_dh) -> np.ndarray:
    """Trilinear groups [n][5][N]^3 from a periodic coarse field [5][cn]^3;
    layout int32 [n][4] = (level, ox, oy, oz)."""
    coarse = _f64(coarse)
    layout = np.ascontiguousarray(layout, dtype=np.int32)
    n = layout.shape[0]
    N = 16 + 2 * g
    out = np.empty((n, 5, N, N, N))
    _lib().oracle_fill_groups_interp(_p(coarse), coarse.shape[1], _p(layout), n, g, base_dh, _p(out))
    return out


def fill_groups_amr(fine, layout, ng0, alpha, coarse0, coarse1, g) -> np.ndarray:
    """AMR preparation step (Sec. 4.2): padded groups [n][5][N]^3 from the
    groups' own interiors fine [n][5][16]^3, same-level neighbours where they
    cover a ghost cell, else the coarse pair blended at alpha[level] and
    interpolated trilinearly; layout int32 [n][4] = (level, ox, oy, oz)."""
    fine = _f64(fine)
    c0, c1 = _f64(coarse0), _f64(coarse1)
    layout = np.ascontiguousarray(layout, dtype=np.int32)
    alpha = _f64(np.asarray(alpha, dtype=np.float64))
    n = layout.shape[0]
    N = 16 + 2 * g
    out = np.empty((n, 5, N, N, N))
    rc = _lib().oracle_fill_groups_amr(_p(fine), _p(layout), n, ng0, alpha.shape[0], _p(c0), _p(c1), c0.shape[1],
                                       _p(alpha), g, _p(out))
    if rc != 0:
        raise ValueError("bad AMR layout or sizes")
    return out


def amr_correct(coarse, shape, cflux, fine, flayout, fflux, dt, dh) -> np.ndarray:
    """Coarse-grid correction after a coarse step (refluxing at coarse-fine
    faces, then restriction of the refined patches); returns the corrected
    copy of the coarse box [Gc][5][16]^3 (patch-group order, shape = (nx, ny,
    nz)).  cflux [Gc][3][3][5][16][16] (with mid planes), fine [nf][5][16]^3
    on the fine grid (ratio 2), flayout int32 [nf][4] (unused, ox, oy, oz),
    fflux [nf][3][2][5][16][16] averaged over the fine sub-steps."""
    out = _f64(coarse).copy()
    cf, fi, ff = _f64(cflux), _f64(fine), _f64(fflux)
    lay = np.ascontiguousarray(flayout, dtype=np.int32)
    nx, ny, nz = shape
    rc = _lib().oracle_amr_correct(_p(out), nx, ny, nz, _p(cf), _p(fi), _p(lay), lay.shape[0], _p(ff), dt, dh)
    if rc != 0:
        raise ValueError("fine groups must cover whole coarse patches inside the coarse box")
    return out


def cfl_dt(U, dh, gamma, cfl) -> float:
    """dt = cfl*dh / max_cells max_d(|v_d| + c); U is [..., 5, cells...] blocks."""
    U = _f64(U)
    if U.ndim == 4:
        nb, ncell = 1, U[0].size
    else:
        nb, ncell = U.shape[0], U[0, 0].size
    return _lib().oracle_cfl_dt(_p(U), nb, ncell, dh, gamma, cfl)


def conserved_sums(U, dh) -> np.ndarray:
    U = _f64(U)
    if U.ndim == 4:
        nb, ncell = 1, U[0].size
    else:
        nb, ncell = U.shape[0], U[0, 0].size
    s = np.empty(5)
    _lib().oracle_conserved_sums(_p(U), nb, ncell, dh, _p(s))
    return s


def riemann_flux(WL, WR, d, gamma, riemann, flags=0) -> np.ndarray:
    WL, WR = _f64(WL), _f64(WR)
    F = np.empty(5)
    rc = _lib().oracle_riemann_flux(_p(WL), _p(WR), d, gamma, riemann, flags, _p(F))
    if rc != 0:
        raise ValueError("oracle_riemann_flux failed")
    return F


def roe_ok(WL, WR, gamma) -> bool:
    return bool(_lib().oracle_roe_ok(_p(_f64(WL)), _p(_f64(WR)), gamma))


def exact_riemann(WL, WR, gamma, xi=()):
    """Exact Riemann problem along x: (star dict, W[len(xi)][5])."""
    WL, WR = _f64(WL), _f64(WR)
    xi = _f64(np.atleast_1d(np.asarray(xi, dtype=np.float64)))
    star = np.empty(5)
    W = np.empty((max(len(xi), 1), 5))
    _lib().oracle_exact_riemann(_p(WL), _p(WR), gamma, _p(star), _p(xi), len(xi), _p(W))
    return ({"p": star[0], "u": star[1], "rhoL": star[2], "rhoR": star[3], "ok": bool(star[4])},
            W[:len(xi)])


def limiter(dl, dr, lim) -> float:
    return _lib().oracle_limiter(float(dl), float(dr), lim)


def slope(wm, w0, wp, d, gamma, lim, flags=0) -> np.ndarray:
    s = np.empty(5)
    _lib().oracle_slope(_p(_f64(wm)), _p(_f64(w0)), _p(_f64(wp)), d, gamma, lim, flags, _p(s))
    return s


def ppm_edge(wa, wb, sa, sb) -> np.ndarray:
    e = np.empty(5)
    _lib().oracle_ppm_edge(_p(_f64(wa)), _p(_f64(wb)), _p(_f64(sa)), _p(_f64(sb)), _p(e))
    return e


def ctu_trace(w, wl, wr, ppm, dtdh, gamma):
    """CTU characteristic tracing of one cell in its direction's frame
    (normal velocity first): returns the half-step states (left face, right
    face) from the cell state w and its reconstructed face values wl, wr."""
    ol, orr = np.empty(5), np.empty(5)
    _lib().oracle_ctu_trace(_p(_f64(w)), _p(_f64(wl)), _p(_f64(wr)), int(ppm), dtdh, gamma, _p(ol), _p(orr))
    return ol, orr


def ppm_monotonize(w, wl, wr):
    """PPM parabola monotonization of one cell: returns the new (wl, wr)."""
    a, b = _f64(wl).copy(), _f64(wr).copy()
    _lib().oracle_ppm_monotonize(_p(_f64(w)), _p(a), _p(b))
    return a, b


def char_roundtrip(w, dw, gamma):
    """(L dw, R L dw) at frame-ordered state w."""
    a, b = np.empty(5), np.empty(5)
    _lib().oracle_char(_p(_f64(w)), _p(_f64(dw)), gamma, _p(a), _p(b))
    return a, b


def stats(counting=False) -> dict:
    s = (ctypes.c_longlong * 4)()
    _lib(counting).oracle_get_stats(ctypes.cast(s, ctypes.c_void_p))
    return {"solves": s[0], "roe_fail": s[1], "floor_hits": s[2], "exact_fail": s[3]}


def reset_stats(counting=False) -> None:
    _lib(counting).oracle_reset_stats()


def ops() -> int:
    return int(_lib(True).oracle_get_ops())


def reset_ops() -> None:
    _lib(True).oracle_reset_ops()

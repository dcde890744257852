"""Python binding of the C ABI in include/hydro.h (ctypes; argument
marshalling only -- every step of the solver runs in the HIP library).

Device buffers are torch tensors on a HIP device; the current torch stream is
passed to every call.  The library must be built
(``python -m paper_1103_3373_amd.build``); if ``libhydro.so`` is missing or
cannot be loaded, every call raises -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhydro.so")

MHM, VL, CTU = 0, 1, 2
PLM, PPM = 0, 1
ROE, HLLC, HLLE, EXACT = 0, 1, 2, 3
GMINMOD, VANLEER, VANALBADA, HYBRID = 0, 1, 2, 3
F64, CHAR, FLUX_MID, PLAIN, ROE_FB_HLLC, BOX_GROUPED, BOX_SEGS, ROE_FB_EXACT = 0x01, 0x02, 0x04, 0x08, 0x10, 0x20, \
    0x40, 0x80
NOALLOC_MAX_GROUPS = 1 << 20  # HYDRO_NOALLOC_MAX_GROUPS

EXPORTS = (
    "hydro_ghost_width", "hydro_solve_groups", "hydro_cfl_dt", "hydro_conserved_sums", "hydro_cfl_dt_sums",
    "hydro_fill_ghosts_periodic", "hydro_fill_groups_interp", "hydro_group_map_len", "hydro_build_group_map",
    "hydro_fill_groups_amr", "hydro_amr_correct", "hydro_accumulate", "hydro_solve_batch", "hydro_autotune",
    "hydro_set_launch_shape", "hydro_get_launch_shape", "hydro_step_box", "hydro_cfl_dt_batch", "hydro_cfl_dt_batch_noalloc",
    "hydro_get_diag", "hydro_last_error", "hydro_shutdown",
)


class HydroError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed ({code}): {msg}")
        self.code = code


class Seg(ctypes.Structure):
    _fields_ = [("in_", ctypes.c_void_p), ("out", ctypes.c_void_p), ("flux", ctypes.c_void_p),
                ("dt", ctypes.c_void_p), ("dt_scale", ctypes.c_double), ("dh", ctypes.c_double),
                ("first", ctypes.c_longlong), ("count", ctypes.c_longlong),
                ("ngx", ctypes.c_int), ("ngy", ctypes.c_int), ("ngz", ctypes.c_int), ("box", ctypes.c_int)]


class Spec(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("reconstruction", ctypes.c_int), ("riemann", ctypes.c_int),
                ("limiter", ctypes.c_int), ("flags", ctypes.c_int), ("gamma", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("roe_fallbacks", ctypes.c_ulonglong), ("floor_hits", ctypes.c_ulonglong)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhydro.so (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run python -m paper_1103_3373_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, i, d, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    L.hydro_ghost_width.argtypes = [i, i]
    L.hydro_ghost_width.restype = i
    L.hydro_solve_groups.argtypes = [P, P, P, i, d, d, d, i, i, i, i, i, P]
    L.hydro_solve_groups.restype = i
    L.hydro_cfl_dt.argtypes = [P, i, d, d, d, i, P, P]
    L.hydro_cfl_dt.restype = i
    L.hydro_conserved_sums.argtypes = [P, i, d, i, P, P]
    L.hydro_cfl_dt_sums.argtypes = [P, i, d, d, d, i, P, P, P]
    L.hydro_cfl_dt_sums.restype = i
    L.hydro_conserved_sums.restype = i
    L.hydro_fill_ghosts_periodic.argtypes = [P, i, i, i, i, i, P, P]
    L.hydro_fill_ghosts_periodic.restype = i
    L.hydro_fill_groups_interp.argtypes = [P, i, P, i, i, d, i, P, P]
    L.hydro_fill_groups_interp.restype = i
    L.hydro_group_map_len.argtypes = [i, i]
    L.hydro_group_map_len.restype = ll
    L.hydro_build_group_map.argtypes = [P, i, i, i, P, P]
    L.hydro_build_group_map.restype = i
    L.hydro_fill_groups_amr.argtypes = [P, P, i, P, i, i, P, P, i, ctypes.POINTER(d), i, i, P, P]
    L.hydro_fill_groups_amr.restype = i
    L.hydro_amr_correct.argtypes = [P, i, P, P, P, i, P, P, d, d, i, P]
    L.hydro_amr_correct.restype = i
    L.hydro_accumulate.argtypes = [P, P, d, ll, i, P]
    L.hydro_accumulate.restype = i
    L.hydro_step_box.argtypes = [P, P, P, i, i, i, P, d, d, d, i, i, i, i, i, P]
    L.hydro_step_box.restype = i
    L.hydro_cfl_dt_batch.argtypes = [P, i, ll, d, d, i, P]
    L.hydro_cfl_dt_batch.restype = i
    L.hydro_cfl_dt_batch_noalloc.argtypes = [P, i, ll, d, d, i, P]
    L.hydro_cfl_dt_batch_noalloc.restype = i
    L.hydro_solve_batch.argtypes = [P, i, ll, ctypes.POINTER(Spec), P]
    L.hydro_solve_batch.restype = i
    L.hydro_autotune.argtypes = [ctypes.POINTER(Spec), i, P]
    L.hydro_autotune.restype = i
    L.hydro_set_launch_shape.argtypes = [ctypes.POINTER(Spec), i, i, i]
    L.hydro_set_launch_shape.restype = i
    L.hydro_get_launch_shape.argtypes = [ctypes.POINTER(Spec), i, i, i, P, P, P]
    L.hydro_get_launch_shape.restype = i
    L.hydro_get_diag.argtypes = [ctypes.POINTER(Diag), i, P]
    L.hydro_get_diag.restype = i
    L.hydro_last_error.argtypes = []
    L.hydro_last_error.restype = ctypes.c_char_p
    L.hydro_shutdown.argtypes = []
    L.hydro_shutdown.restype = None
    _lib = L
    return L


def _check(fn: str, rc: int) -> int:
    if rc < 0:
        raise HydroError(fn, rc, lib().hydro_last_error().decode())
    return rc


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _dtype_flag(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return 0
    raise TypeError(f"unsupported dtype {t.dtype}")


def _require(t: torch.Tensor, name: str, shape=None, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def ghost_width(scheme: int, recon: int) -> int:
    return _check("hydro_ghost_width", lib().hydro_ghost_width(scheme, recon))


def solve_groups(inp, out, flux=None, *, dt, dh, gamma, scheme, recon, riemann, limiter=VANLEER, char=False,
                 plain=False, flux_mid=False, roe_fb_hllc=False, roe_fb_exact=False, stream=None):
    """One step of n patch groups: inp [n,5,N,N,N] -> out [n,5,16,16,16].
    riemann=EXACT and roe_fb_exact run on the plain path."""
    n = inp.shape[0]
    N = 16 + 2 * ghost_width(scheme, recon)
    _require(inp, "inp", (n, 5, N, N, N))
    _require(out, "out", (n, 5, 16, 16, 16), inp.dtype)
    if flux is not None:
        _require(flux, "flux", (n, 3, 3 if flux_mid else 2, 5, 16, 16), inp.dtype)
    flags = _dtype_flag(inp) | (CHAR if char else 0) | (PLAIN if plain else 0) | (FLUX_MID if flux_mid else 0) \
        | (ROE_FB_HLLC if roe_fb_hllc else 0) | (ROE_FB_EXACT if roe_fb_exact else 0)
    _check("hydro_solve_groups", lib().hydro_solve_groups(
        _ptr(inp), _ptr(out), _ptr(flux), n, float(dt), float(dh), float(gamma), scheme, recon, riemann, limiter,
        flags, _stream(stream)))
    return out


def cfl_dt(U, dh, gamma, cfl, dt_out=None, stream=None):
    """FP64 dt from interiors U [n,5,16,16,16] into a device double tensor."""
    _require(U, "U")
    if dt_out is None:
        dt_out = torch.empty(1, dtype=torch.float64, device=U.device)
    _check("hydro_cfl_dt", lib().hydro_cfl_dt(_ptr(U), U.shape[0], float(dh), float(gamma), float(cfl),
                                              _dtype_flag(U), _ptr(dt_out), _stream(stream)))
    return dt_out


def conserved_sums(U, dh, sums_out=None, stream=None):
    _require(U, "U")
    if sums_out is None:
        sums_out = torch.empty(5, dtype=torch.float64, device=U.device)
    _check("hydro_conserved_sums", lib().hydro_conserved_sums(_ptr(U), U.shape[0], float(dh), _dtype_flag(U),
                                                              _ptr(sums_out), _stream(stream)))
    return sums_out


def cfl_dt_sums(U, dh, gamma, cfl, dt_out=None, sums_out=None, stream=None):
    """FP64 dt and conserved sums of interiors U [n,5,16,16,16] in one pass
    (bit-identical to cfl_dt and conserved_sums)."""
    _require(U, "U")
    if dt_out is None:
        dt_out = torch.empty(1, dtype=torch.float64, device=U.device)
    if sums_out is None:
        sums_out = torch.empty(5, dtype=torch.float64, device=U.device)
    _check("hydro_cfl_dt_sums", lib().hydro_cfl_dt_sums(_ptr(U), U.shape[0], float(dh), float(gamma), float(cfl),
                                                        _dtype_flag(U), _ptr(dt_out), _ptr(sums_out),
                                                        _stream(stream)))
    return dt_out, sums_out


def fill_ghosts_periodic(box, g, out=None, *, grouped=False, shape=None, stream=None):
    """Ghosted groups from a periodic box [5,nz,ny,nx] (or grouped [G,5,16,16,16]
    with shape=(nx, ny, nz))."""
    _require(box, "box")
    if grouped:
        nx, ny, nz = shape
    else:
        _, nz, ny, nx = box.shape
    N = 16 + 2 * g
    G = (nx // 16) * (ny // 16) * (nz // 16)
    if out is None:
        out = torch.empty((G, 5, N, N, N), dtype=box.dtype, device=box.device)
    _require(out, "out", (G, 5, N, N, N), box.dtype)
    flags = _dtype_flag(box) | (BOX_GROUPED if grouped else 0)
    _check("hydro_fill_ghosts_periodic", lib().hydro_fill_ghosts_periodic(_ptr(box), nx, ny, nz, g, flags,
                                                                          _ptr(out), _stream(stream)))
    return out


def fill_groups_interp(coarse, layout, g, base_dh, out=None, stream=None):
    """AMR-shaped groups by trilinear interpolation of coarse [5,cn,cn,cn];
    layout int32 [n,4] = (level, ox, oy, oz)."""
    _require(coarse, "coarse")
    _require(layout, "layout", dtype=torch.int32)
    n = layout.shape[0]
    N = 16 + 2 * g
    if out is None:
        out = torch.empty((n, 5, N, N, N), dtype=coarse.dtype, device=coarse.device)
    _check("hydro_fill_groups_interp", lib().hydro_fill_groups_interp(
        _ptr(coarse), coarse.shape[1], _ptr(layout), n, g, float(base_dh), _dtype_flag(coarse), _ptr(out),
        _stream(stream)))
    return out


def group_map_len(ng0, n_levels) -> int:
    n = lib().hydro_group_map_len(int(ng0), int(n_levels))
    if n < 0:
        raise ValueError(f"bad AMR level sizes ng0={ng0}, n_levels={n_levels}")
    return n


def build_group_map(layout, ng0, n_levels, out=None, stream=None):
    """Per-level map from group position to group index (-1 where none);
    layout int32 [n,4] = (level, ox, oy, oz) on the device."""
    _require(layout, "layout", dtype=torch.int32)
    m = group_map_len(ng0, n_levels)
    if out is None:
        out = torch.empty((m,), dtype=torch.int32, device=layout.device)
    _require(out, "map", shape=(m,), dtype=torch.int32)
    _check("hydro_build_group_map", lib().hydro_build_group_map(
        _ptr(layout), layout.shape[0], int(ng0), int(n_levels), _ptr(out), _stream(stream)))
    return out


def fill_groups_amr(fine, layout, gmap, ng0, alpha, coarse0, coarse1, g, out=None, stream=None):
    """Preparation step with spatial and temporal interpolation: padded groups
    [n,5,N,N,N] from the groups' interiors fine [n,5,16,16,16], same-level
    neighbours (gmap from build_group_map) and the coarse pair blended at
    alpha[level] (a host sequence, one weight per level)."""
    _require(fine, "fine")
    _require(layout, "layout", dtype=torch.int32)
    _require(gmap, "map", dtype=torch.int32)
    _require(coarse0, "coarse0", dtype=fine.dtype)
    _require(coarse1, "coarse1", shape=coarse0.shape, dtype=fine.dtype)
    n = layout.shape[0]
    if tuple(fine.shape) != (n, 5, 16, 16, 16):
        raise ValueError(f"fine has shape {tuple(fine.shape)}, expected {(n, 5, 16, 16, 16)}")
    if gmap.shape[0] != group_map_len(ng0, len(alpha)):
        raise ValueError("map length does not match ng0 and the level count")
    N = 16 + 2 * g
    if out is None:
        out = torch.empty((n, 5, N, N, N), dtype=fine.dtype, device=fine.device)
    _require(out, "out", shape=(n, 5, N, N, N), dtype=fine.dtype)
    al = (ctypes.c_double * len(alpha))(*[float(x) for x in alpha])
    _check("hydro_fill_groups_amr", lib().hydro_fill_groups_amr(
        _ptr(fine), _ptr(layout), n, _ptr(gmap), int(ng0), len(alpha), _ptr(coarse0), _ptr(coarse1),
        coarse0.shape[1], al, g, _dtype_flag(fine), _ptr(out), _stream(stream)))
    return out


def amr_correct(coarse, n, coarse_flux, fine, fine_layout, fine_map, fine_flux, dt, dh, stream=None):
    """Coarse-grid correction in place on the coarse box [G,5,16,16,16]
    (patch-group order, n^3 cells): refluxing at the coarse-fine faces, then
    restriction of the refined patches."""
    G = (n // 16) ** 3
    nf = fine_layout.shape[0]
    _require(coarse, "coarse", (G, 5, 16, 16, 16))
    _require(coarse_flux, "coarse_flux", (G, 3, 3, 5, 16, 16), coarse.dtype)
    _require(fine, "fine", (nf, 5, 16, 16, 16), coarse.dtype)
    _require(fine_layout, "fine_layout", dtype=torch.int32)
    _require(fine_map, "fine_map", (group_map_len(n // 8, 1),), torch.int32)
    _require(fine_flux, "fine_flux", (nf, 3, 2, 5, 16, 16), coarse.dtype)
    _check("hydro_amr_correct", lib().hydro_amr_correct(
        _ptr(coarse), n, _ptr(coarse_flux), _ptr(fine), _ptr(fine_layout), nf, _ptr(fine_map), _ptr(fine_flux),
        float(dt), float(dh), _dtype_flag(coarse), _stream(stream)))
    return coarse


def accumulate(acc, x, w, stream=None):
    """acc += w * x elementwise (evaluated in FP64)."""
    _require(acc, "acc")
    _require(x, "x", tuple(acc.shape), acc.dtype)
    _check("hydro_accumulate", lib().hydro_accumulate(_ptr(acc), _ptr(x), float(w), acc.numel(),
                                                      _dtype_flag(acc), _stream(stream)))
    return acc


def make_spec(scheme, recon, riemann, limiter=VANLEER, *, gamma, char=False, f64=False, flux_mid=False,
              roe_fb_hllc=False, box_segs=False) -> Spec:
    """box_segs: the batch's segments are all periodic boxes (HYDRO_BOX_SEGS)."""
    flags = (F64 if f64 else 0) | (CHAR if char else 0) | (FLUX_MID if flux_mid else 0) \
        | (ROE_FB_HLLC if roe_fb_hllc else 0) | (BOX_SEGS if box_segs else 0)
    return Spec(scheme, recon, riemann, limiter, flags, float(gamma))


def seg_table(segs, device) -> torch.Tensor:
    """Pack hydro_seg records into a device byte tensor.  Each record is
    (in, out, flux|None, dt_tensor, dt_scale, dh, first, count) for ghosted
    groups, or with a trailing (ngx, ngy, ngz) for a periodic grouped box."""
    arr = (Seg * len(segs))()
    for q, rec in enumerate(segs):
        i, o, f, dtt, sc, dh, first, count = rec[:8]
        box = rec[8] if len(rec) > 8 else None
        arr[q] = Seg(i.data_ptr(), o.data_ptr(), 0 if f is None else f.data_ptr(), dtt.data_ptr(), float(sc),
                     float(dh), int(first), int(count), *(box if box else (0, 0, 0)), 1 if box else 0)
    host = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    if torch.device(device).type == "cuda":
        # pinned + non-blocking: the host does not wait for the device
        return host.pin_memory().to(device, non_blocking=True)
    return host.to(device)


def step_box(box_in, box_out, shape, dt_dev, *, dh, gamma, scheme, recon, riemann, limiter=VANLEER, char=False,
             dt_scale=1.0, flux=None, flux_mid=False, roe_fb_hllc=False, stream=None):
    """One step of a periodic box in patch-group order [G,5,16,16,16]
    (shape = (nx, ny, nz)); dt is read from the device double dt_dev."""
    nx, ny, nz = shape
    G = (nx // 16) * (ny // 16) * (nz // 16)
    _require(box_in, "box_in", (G, 5, 16, 16, 16))
    _require(box_out, "box_out", (G, 5, 16, 16, 16), box_in.dtype)
    _require(dt_dev, "dt_dev", dtype=torch.float64)
    flags = _dtype_flag(box_in) | (CHAR if char else 0) | (FLUX_MID if flux_mid else 0) \
        | (ROE_FB_HLLC if roe_fb_hllc else 0)
    _check("hydro_step_box", lib().hydro_step_box(_ptr(box_in), _ptr(box_out), _ptr(flux), nx, ny, nz,
                                                  _ptr(dt_dev), float(dt_scale), float(dh), float(gamma), scheme,
                                                  recon, riemann, limiter, flags, _stream(stream)))
    return box_out


def solve_batch(seg_dev: torch.Tensor, n_segs: int, n_groups_total: int, spec: Spec, stream=None):
    _check("hydro_solve_batch", lib().hydro_solve_batch(_ptr(seg_dev), n_segs, int(n_groups_total),
                                                        ctypes.byref(spec), _stream(stream)))


def cfl_dt_batch(seg_dev: torch.Tensor, n_segs: int, n_groups_total: int, *, gamma, cfl, f64=False, stream=None):
    """FP64 dt of every segment's `out` state, written to its dt pointer."""
    _check("hydro_cfl_dt_batch", lib().hydro_cfl_dt_batch(_ptr(seg_dev), n_segs, int(n_groups_total), float(gamma),
                                                          float(cfl), F64 if f64 else 0, _stream(stream)))


def cfl_dt_batch_noalloc(seg_dev: torch.Tensor, n_segs: int, n_groups_total: int, *, gamma, cfl, f64=False,
                         stream=None):
    """cfl_dt_batch without device allocation (library-owned static scratch of
    NOALLOC_MAX_GROUPS groups; calls that overlap in time on one device race)."""
    _check("hydro_cfl_dt_batch_noalloc",
           lib().hydro_cfl_dt_batch_noalloc(_ptr(seg_dev), n_segs, int(n_groups_total), float(gamma), float(cfl),
                                            F64 if f64 else 0, _stream(stream)))


def autotune(spec: Spec, n_groups_hint: int, stream=None) -> int:
    return _check("hydro_autotune", lib().hydro_autotune(ctypes.byref(spec), int(n_groups_hint), _stream(stream)))


def set_launch_shape(spec: Spec, grid: int, variant: int, zrun: int = 0) -> None:
    """Pin the fused kernel's launch shape for spec's specialization
    (grid 0 = default; variant 2 or 4; zrun = groups per z-run of a box
    step, 0 = default; see hydro_set_launch_shape)."""
    _check("hydro_set_launch_shape", lib().hydro_set_launch_shape(ctypes.byref(spec), int(grid), int(variant),
                                                                  int(zrun)))


def get_launch_shape(spec: Spec, shape) -> tuple:
    """(grid, variant, zrun) that step_box uses for spec on a box of
    shape = (nx, ny, nz) without flux output."""
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    nx, ny, nz = shape
    _check("hydro_get_launch_shape", lib().hydro_get_launch_shape(ctypes.byref(spec), int(nx), int(ny), int(nz),
                                                                  ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def get_diag(reset=False, stream=None) -> dict:
    d = Diag()
    _check("hydro_get_diag", lib().hydro_get_diag(ctypes.byref(d), 1 if reset else 0, _stream(stream)))
    return {"roe_fallbacks": int(d.roe_fallbacks), "floor_hits": int(d.floor_hits)}


def shutdown():
    lib().hydro_shutdown()

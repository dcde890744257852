"""The allocation-free batched time step (hydro_cfl_dt_batch_noalloc) against
hydro_cfl_dt_batch, through the C ABI: bit-identical time steps on two calls
in a row, the second with a smaller batch (fewer segments and groups), so
stale per-group maxima of the first call would show; both also equal the
oracle's FP64 time step of each simulation (max is order-free and both sides
evaluate the same uncontracted expression)."""
import ctypes

import numpy as np
import pytest

import oracle as O
from paper_1103_3373_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _table(H, boxes, dtype):
    """Segment table whose `out` states are the given boxes (grouped)."""
    rows, keep, first = [], [], 0
    for box in boxes:
        n = box.shape[-1]
        g = torch.from_numpy(W.box_to_groups(box)).to(device="cuda", dtype=dtype)
        dt = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        ng = n // 16
        rows.append((g, g, None, dt, 1.0, 1.0 / n, first, g.shape[0], (ng, ng, ng)))
        keep.append((g, dt))
        first += g.shape[0]
    return H.seg_table(rows, "cuda"), len(rows), first, keep


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_dt_equals_allocating_dt(dtype):
    from paper_1103_3373_amd import hydro as H
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    gamma, cfl = 1.4, 0.4
    f64 = dtype == torch.float64
    big = [W.lognormal_blast_box(64, gamma=gamma, seed=11, radius_cells=4), W.sod_box(32, gamma=gamma, seed=12),
           W.blast_box(48, gamma=gamma, seed=13, radius_cells=3), W.kelvin_helmholtz_box(32, gamma=gamma)]
    small = [W.blast_box(32, gamma=gamma, seed=21, radius_cells=2), W.sod_box(16, gamma=gamma, seed=22)]
    for boxes in (big, small):
        table, n_segs, total, keep = _table(H, boxes, dtype)
        H.cfl_dt_batch(table, n_segs, total, gamma=gamma, cfl=cfl, f64=f64)
        torch.cuda.synchronize()
        want = [dt.item() for _, dt in keep]
        for _, dt in keep:
            dt.fill_(-1.0)
        # The raw C entry point, as a caller that cannot allocate would call it.
        rc = H.lib().hydro_cfl_dt_batch_noalloc(ctypes.c_void_p(table.data_ptr()), n_segs, ctypes.c_longlong(total),
                                                gamma, cfl, H.F64 if f64 else 0,
                                                ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == 0, H.lib().hydro_last_error()
        torch.cuda.synchronize()
        got = [dt.item() for _, dt in keep]
        assert got == want
        for (g, _), box, dt in zip(keep, boxes, got):
            state = g.cpu().numpy().astype(np.float64)
            assert dt == O.cfl_dt(state, 1.0 / box.shape[-1], gamma, cfl)
    with pytest.raises(H.HydroError):
        H.cfl_dt_batch_noalloc(table, n_segs, H.NOALLOC_MAX_GROUPS + 1, gamma=gamma, cfl=cfl, f64=f64)

"""Precision on smooth data: a Kelvin-Helmholtz shear layer (tanh interfaces
of width 4 cells) advanced 100 steps by the FP32 and FP64 GPU paths and by
the FP64 oracle on the same time-step sequence, for MHM, VL and CTU
(PPM with characteristic limiting + HLLC); FP64 conservation sums on the GPU.

Errors are L1 norms of the difference per conserved variable, relative to
the reference's L1 norm of that variable; the momentum components share
the momentum magnitude |m| as scale (the z momentum of this flow is zero
everywhere and the y momentum is a small perturbation).

Bars: FP32 GPU vs oracle <= 1e-5; FP64 GPU vs oracle <= 1e-12 after 100
steps; drift of the FP64 conserved sums of mass and energy <= 1e-13
(FP64 path) and <= 1e-6 (FP32 path) relative, of the momenta relative to
the integral of |m|."""
import numpy as np
import pytest

import oracle as O
from paper_1103_3373_amd import workloads as W

from tests._util import field_errors

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 32
STEPS = 100


@pytest.mark.parametrize("scheme,cfl", [(0, 0.3), (1, 0.3), (2, 0.5)])
def test_kelvin_helmholtz_100_steps(scheme, cfl):
    from paper_1103_3373_amd import hydro as H
    gamma = 1.4
    box = W.kelvin_helmholtz_box(N, gamma=gamma)
    grp = W.box_to_groups(box)
    kw = dict(dh=1.0 / N, gamma=gamma, scheme=scheme, recon=H.PPM, riemann=H.HLLC, char=True)
    s64 = torch.from_numpy(grp).cuda()
    s32 = torch.from_numpy(grp.astype(np.float32)).cuda()
    o64, o32 = torch.empty_like(s64), torch.empty_like(s32)
    dt_dev = torch.empty(1, dtype=torch.float64, device="cuda")
    sums0 = H.conserved_sums(s64, 1.0 / N).cpu().numpy()
    ref = box.copy()
    for _ in range(STEPS):
        dt = O.cfl_dt(ref, 1.0 / N, gamma, cfl)
        ref = O.step_box(ref, dt, 1.0 / N, gamma, scheme, 1, 1, 1, O.F_CHAR)
        dt_dev.fill_(dt)
        H.step_box(s64, o64, (N, N, N), dt_dev, **kw)
        H.step_box(s32, o32, (N, N, N), dt_dev, **kw)
        s64, o64 = o64, s64
        s32, o32 = o32, s32
    torch.cuda.synchronize()
    refg = W.box_to_groups(ref)
    e32 = field_errors(s32.cpu().numpy(), refg)[0]
    e64 = field_errors(s64.cpu().numpy(), refg)[0]
    print(f"scheme {scheme}: FP32 rel L1 {e32}, FP64 rel L1 {e64}")
    assert e32.max() <= 1e-5, e32
    assert e64.max() <= 1e-12, e64
    s64n = H.conserved_sums(s64, 1.0 / N).cpu().numpy()
    s32n = H.conserved_sums(s32, 1.0 / N).cpu().numpy()
    for v in (0, 1, 4):
        assert abs(s64n[v] - sums0[v]) <= 1e-13 * abs(sums0[v])
        assert abs(s32n[v] - sums0[v]) <= 1e-6 * abs(sums0[v])
    mom = np.sqrt((grp[:, 1:4] ** 2).sum(1)).sum() / N ** 3  # integral of |m|
    for v in (1, 2, 3):
        assert abs(s64n[v] - sums0[v]) <= 1e-13 * mom
        assert abs(s32n[v] - sums0[v]) <= 1e-6 * mom

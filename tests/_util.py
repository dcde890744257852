"""Shared test helpers (no solver arithmetic)."""
import numpy as np

from paper_1103_3373_amd import workloads as W


def random_smooth_box(n, gamma, seed, amp=0.2, ny=None, nz=None):
    """Smooth positive random state (a few low Fourier modes) on a periodic box."""
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    fields = []
    for _ in range(5):
        f = np.zeros_like(X)
        for _ in range(3):
            k = rng.integers(-2, 3, size=3)
            ph = rng.uniform(0, 2 * np.pi)
            f += rng.uniform(-1, 1) * np.cos(2 * np.pi * (k[0] * X + k[1] * Y + k[2] * Z) + ph)
        fields.append(f)
    rho = 1.0 + amp * fields[0] / 3
    p = 1.0 + amp * fields[4] / 3
    return W.primitive_to_conserved(rho, amp * fields[1], amp * fields[2], amp * fields[3], p, gamma)


def rel_errors(a, b, axis=None):
    """Per-variable (rel_L1, rel_Linf) of a against reference b; arrays [..., 5, ...]
    with the variable on axis 1 (groups) or 0 (box), or on `axis`."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ax = axis if axis is not None else (1 if a.ndim in (5, 6) else 0)
    a = np.moveaxis(a, ax, 0).reshape(5, -1) if a.shape[ax] == 5 else a.reshape(1, -1)
    b = np.moveaxis(b, ax, 0).reshape(5, -1) if b.shape[ax] == 5 else b.reshape(1, -1)
    d = np.abs(a - b)
    l1 = d.sum(1) / np.maximum(np.abs(b).sum(1), 1e-300)
    linf = d.max(1) / np.maximum(np.abs(b).max(1), 1e-300)
    return l1, linf


def scaled_max_err(a, b):
    """max |a-b| / max |b| over the whole array (one number)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def var_max_err(a, b):
    """Largest per-variable max |a-b| of states a against reference b, each
    variable against its own scale: max |rho| for mass, max |E| for energy,
    and the reference's largest momentum magnitude |m| for the three momentum
    components (so a component that is near zero everywhere is not measured
    against the energy).  States grouped [n, 5, ...] or box [5, ...]."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ax = 1 if a.ndim == 5 else 0
    a = np.moveaxis(a, ax, 0).reshape(5, -1)
    b = np.moveaxis(b, ax, 0).reshape(5, -1)
    d = np.abs(a - b).max(axis=1)
    mag = np.sqrt((b[1:4] ** 2).sum(0)).max()
    scale = np.array([np.abs(b[0]).max(), mag, mag, mag, np.abs(b[4]).max()])
    return float((d / np.maximum(scale, 1e-300)).max())


def field_errors(a, b):
    """Per-variable (L1, Linf) error of state a against reference b, both
    grouped [n, 5, 16, 16, 16] or box [5, ...].  Mass and energy errors are
    relative to the reference's own magnitude; the three momentum components
    share the reference's momentum magnitude |m| as scale, so a component that
    is (close to) zero everywhere does not divide by zero."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    ax = 1 if a.ndim == 5 else 0
    a = np.moveaxis(a, ax, 0).reshape(5, -1)
    b = np.moveaxis(b, ax, 0).reshape(5, -1)
    d = np.abs(a - b)
    mag = np.sqrt((b[1:4] ** 2).sum(0))
    s1 = np.array([np.abs(b[0]).sum()] + [mag.sum()] * 3 + [np.abs(b[4]).sum()])
    si = np.array([np.abs(b[0]).max()] + [mag.max()] * 3 + [np.abs(b[4]).max()])
    return d.sum(1) / np.maximum(s1, 1e-300), d.max(1) / np.maximum(si, 1e-300)


def group_window(box, q, g):
    """The ghosted input of patch group q (width g) of a periodic box
    [5][nz][ny][nx], cut out with periodic index wrap: [5][16+2g]^3.  Group
    order (gz*ngy + gy)*ngx + gx.  Indexing only (no solver arithmetic)."""
    nz, ny, nx = box.shape[1:]
    ngx, ngy = nx // 16, ny // 16
    gx, gy, gz = q % ngx, (q // ngx) % ngy, q // (ngx * ngy)
    ix = np.arange(16 * gx - g, 16 * gx + 16 + g) % nx
    iy = np.arange(16 * gy - g, 16 * gy + 16 + g) % ny
    iz = np.arange(16 * gz - g, 16 * gz + 16 + g) % nz
    return box[:, iz][:, :, iy][:, :, :, ix]

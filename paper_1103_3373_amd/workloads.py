"""Seeded synthetic inputs for the unsplit hydro solver.

This module only *generates inputs*: initial conditions on periodic boxes,
AMR-shaped group placements and serving request streams.  It holds none of
the solver's arithmetic and is shared by the HIP path's tests/benchmark and
by the oracle's tests.  Every generator is deterministic in its seed.

The paper's own workloads (a 3D blast wave, Sec. 5.1, and a cosmological AMR
run, Sec. 5.2) are not reproducible here (no initial conditions are given),
so these seeded fields of the same kind stand in for them.

Arrays are float64 numpy, conserved variables (rho, mx, my, mz, E), layout
[5][nz][ny][nx] with x fastest.  A state is *specified* by its primitive
fields; the conserved form uses the ideal-gas total energy
E = p/(gamma-1) + rho |v|^2 / 2, which defines the initial state.
"""
from __future__ import annotations

import numpy as np

IC_SEED = 1103
ARRIVAL_SEED = 3373


def primitive_to_conserved(rho, vx, vy, vz, p, gamma) -> np.ndarray:
    """Stack primitive fields into a conserved [5][...] float64 array."""
    rho = np.asarray(rho, dtype=np.float64)
    shape = np.broadcast(rho, vx, vy, vz, p).shape
    U = np.empty((5,) + shape)
    U[0] = rho
    U[1] = rho * vx
    U[2] = rho * vy
    U[3] = rho * vz
    U[4] = p / (gamma - 1.0) + 0.5 * rho * (np.asarray(vx) ** 2 + np.asarray(vy) ** 2 + np.asarray(vz) ** 2)
    return U


def cell_centres(n: int) -> np.ndarray:
    return (np.arange(n) + 0.5) / n


def sod_box(n=32, gamma=5.0 / 3.0, seed=IC_SEED, noise=1e-3, ny=None, nz=None) -> np.ndarray:
    """Sod shock tube along x on a periodic box (interface on the face x=0.5).

    rho,p = 1,1 for x<0.5 and 0.125,0.1 for x>0.5, v = 0, and a seeded uniform
    +-noise multiplicative density perturbation per cell.
    """
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    x = cell_centres(n)[None, None, :] * np.ones((nz, ny, 1))
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    if noise:
        rng = np.random.default_rng(seed)
        rho = rho * (1.0 + rng.uniform(-noise, noise, size=rho.shape))
    z = np.zeros_like(rho)
    return primitive_to_conserved(rho, z, z, z, p, gamma)


def gaussian_random_field(n, seed, kmin=1, kmax=8, rng=None) -> np.ndarray:
    """Unit-variance Gaussian random field on a periodic n^3 grid, flat
    amplitude over integer wavevectors 1 <= |k| <= kmax, seeded phases."""
    rng = np.random.default_rng(seed) if rng is None else rng
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kz = k1[:, None, None]
    ky = k1[None, :, None]
    kx = np.fft.rfftfreq(n, d=1.0 / n)[None, None, :]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    mask = (kk >= kmin) & (kk <= kmax)
    spec = (rng.standard_normal(mask.shape) + 1j * rng.standard_normal(mask.shape)) * mask
    f = np.fft.irfftn(spec, s=(n, n, n), axes=(0, 1, 2))
    f -= f.mean()
    s = f.std()
    return f / s if s > 0 else f


def blast_mask(n, seed, n_blasts=4, radius_cells=8, rng=None) -> np.ndarray:
    """Boolean mask of n_blasts seeded spheres (radius in cells, periodic)."""
    rng = np.random.default_rng(seed) if rng is None else rng
    c = np.arange(n) + 0.5
    mask = np.zeros((n, n, n), dtype=bool)
    for _ in range(n_blasts):
        ctr = rng.uniform(0.0, n, size=3)  # (x, y, z) in cells
        dx = np.abs(c - ctr[0]); dx = np.minimum(dx, n - dx)
        dy = np.abs(c - ctr[1]); dy = np.minimum(dy, n - dy)
        dz = np.abs(c - ctr[2]); dz = np.minimum(dz, n - dz)
        r2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        mask |= r2 <= radius_cells * radius_cells
    return mask


def lognormal_blast_box(n=256, gamma=1.4, seed=IC_SEED, sigma=0.5, kmax=8, mach=1.0, blasts=True,
                        p_blast=100.0, radius_cells=8) -> np.ndarray:
    """Lognormal density (sigma 0.5) on a smooth random field with k <= kmax,
    pressure 1, smooth Gaussian velocities with rms |v| = mach * c(<rho>=1),
    plus 4 seeded spherical blasts (p = 100, radius 8 cells)."""
    rng = np.random.default_rng(seed)
    g = gaussian_random_field(n, seed, kmax=kmax, rng=rng)
    rho = np.exp(sigma * g - 0.5 * sigma * sigma)
    vel = [gaussian_random_field(n, seed, kmax=kmax, rng=rng) for _ in range(3)]
    vrms = np.sqrt(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2))
    target = mach * np.sqrt(gamma * 1.0 / 1.0)
    vel = [v * (target / vrms) for v in vel]
    p = np.ones((n, n, n))
    if blasts:
        p[blast_mask(n, seed, radius_cells=radius_cells, rng=rng)] = p_blast
    return primitive_to_conserved(rho, vel[0], vel[1], vel[2], p, gamma)


def blast_box(n, gamma=1.4, seed=IC_SEED, p_blast=100.0, radius_cells=8) -> np.ndarray:
    """Uniform rho=1, p=1 gas at rest with 4 seeded spherical blasts."""
    rng = np.random.default_rng(seed)
    p = np.ones((n, n, n))
    p[blast_mask(n, seed, radius_cells=radius_cells, rng=rng)] = p_blast
    rho = np.ones((n, n, n))
    z = np.zeros((n, n, n))
    return primitive_to_conserved(rho, z, z, z, p, gamma)


def kelvin_helmholtz_box(n=64, gamma=1.4, seed=IC_SEED, width_cells=4.0, amp=0.01, p0=2.5) -> np.ndarray:
    """Smooth shear layer: rho=2, vx=+0.5 inside |y-0.5|<0.25, rho=1, vx=-0.5
    outside, tanh interfaces of width `width_cells` cells, vy = amp sin(4 pi x
    + phase) weighted by the interface profile, p = p0, seeded phase."""
    rng = np.random.default_rng(seed)
    phase = rng.uniform(0.0, 2.0 * np.pi)
    x = cell_centres(n)[None, None, :]
    y = cell_centres(n)[None, :, None]
    w = width_cells / n
    s = 0.5 * (np.tanh((y - 0.25) / w) - np.tanh((y - 0.75) / w))  # 1 inside, 0 outside
    shape = (n, n, n)
    rho = np.broadcast_to(1.0 + s, shape)
    vx = np.broadcast_to(-0.5 + s, shape)
    vy = np.broadcast_to(amp * np.sin(4.0 * np.pi * x + phase) * 4.0 * s * (1.0 - s), shape)
    vz = np.zeros(shape)
    p = np.full(shape, p0)
    return primitive_to_conserved(rho, vx, vy, vz, p, gamma)


def sound_wave_box(nx, ny, nz, gamma=5.0 / 3.0, amp=1e-6, kvec=(1, 1, 1), rho0=1.0, p0=None, t=0.0):
    """Linear sound wave rho = rho0 (1 + amp cos(2 pi k.x - w t)) travelling along k.

    Point values at cell centres.  Returns (U, period)."""
    p0 = 1.0 / gamma if p0 is None else p0  # sound speed 1
    c0 = np.sqrt(gamma * p0 / rho0)
    k = np.asarray(kvec, dtype=np.float64)
    kn = np.linalg.norm(k)
    x = cell_centres(nx)[None, None, :]
    y = cell_centres(ny)[None, :, None]
    z = cell_centres(nz)[:, None, None]
    ph = 2.0 * np.pi * (k[0] * x + k[1] * y + k[2] * z) - 2.0 * np.pi * kn * c0 * t
    d = amp * np.cos(ph) * np.ones((nz, ny, nx))
    rho = rho0 * (1.0 + d)
    vmag = c0 * d
    vx, vy, vz = (vmag * k[i] / kn for i in range(3))
    p = p0 + c0 * c0 * rho0 * d
    period = 1.0 / (kn * c0)
    return primitive_to_conserved(rho, vx, vy, vz, p, gamma), period


def box_to_groups(box: np.ndarray) -> np.ndarray:
    """Re-layout an interior box [5][nz][ny][nx] into patch-group order
    [G][5][16][16][16], G = (gz*ngy + gy)*ngx + gx (a permutation only)."""
    _, nz, ny, nx = box.shape
    b = box.reshape(5, nz // 16, 16, ny // 16, 16, nx // 16, 16)
    return np.ascontiguousarray(b.transpose(1, 3, 5, 0, 2, 4, 6).reshape(-1, 5, 16, 16, 16))


def groups_to_box(groups: np.ndarray, nx: int, ny: int, nz: int) -> np.ndarray:
    """Inverse of box_to_groups."""
    g = groups.reshape(nz // 16, ny // 16, nx // 16, 5, 16, 16, 16)
    return np.ascontiguousarray(g.transpose(3, 0, 4, 1, 5, 2, 6).reshape(5, nz, ny, nx))


# ---------------------------------------------------------------------------
# AMR-shaped batch: distinct seeded patch-group positions on refinement levels
# ---------------------------------------------------------------------------
def amr_layout(level_counts=(2048, 6144, 12288), base_n=256, seed=IC_SEED) -> np.ndarray:
    """Seeded patch-group placements on refinement levels of ratio 2.

    Returns int32 array [n_groups][4] of (level, ox, oy, oz): the level and
    the level-grid index of the group's first interior cell (multiples of 16).
    Level l covers the unit box with base_n * 2^l cells per side."""
    rng = np.random.default_rng(seed)
    rows = []
    for lev, cnt in enumerate(level_counts):
        ng = (base_n << lev) // 16
        total = ng ** 3
        if cnt > total:
            raise ValueError("too many groups for level")
        pick = rng.choice(total, size=cnt, replace=False)
        gz, rem = np.divmod(pick, ng * ng)
        gy, gx = np.divmod(rem, ng)
        rows.append(np.stack([np.full(cnt, lev), gx * 16, gy * 16, gz * 16], axis=1))
    return np.ascontiguousarray(np.concatenate(rows).astype(np.int32))


def amr_coarse_field(n=64, gamma=1.4, seed=IC_SEED) -> np.ndarray:
    """The seeded smooth coarse field that AMR-shaped groups interpolate from
    (lognormal density with blasts, as for the uniform-mesh workload)."""
    return lognormal_blast_box(n, gamma=gamma, seed=seed)


# ---------------------------------------------------------------------------
# Serving stream
# ---------------------------------------------------------------------------
def request_stream(n_requests=2000, rate=200.0, seed=ARRIVAL_SEED, sizes=(32, 64, 128),
                   schemes=(0, 1, 2), riemanns=(0, 1), ics=("sod", "blast", "lognormal")):
    """Poisson arrivals; each request draws box size, scheme, solver and IC
    uniformly.  Returns a list of dicts sorted by arrival time (seconds)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for q in range(n_requests):
        out.append({
            "id": q,
            "arrival": float(t[q]),
            "n": int(rng.choice(sizes)),
            "scheme": int(rng.choice(schemes)),
            "riemann": int(rng.choice(riemanns)),
            "ic": str(rng.choice(ics)),
            "seed": int(rng.integers(0, 2**31 - 1)),
        })
    return out


def initial_box(ic: str, n: int, gamma: float, seed: int) -> np.ndarray:
    if ic == "sod":
        return sod_box(n, gamma=gamma, seed=seed)
    if ic == "blast":
        return blast_box(n, gamma=gamma, seed=seed)
    if ic == "lognormal":
        return lognormal_blast_box(n, gamma=gamma, seed=seed, blasts=False)
    raise ValueError(ic)

"""Seeded synthetic inputs: velocity models, wavelets, initial fields, acquisition
geometry.

This module holds none of the solver's arithmetic (no stencil weights, no
Laplacian, no stability limit, no damping): it only draws and shapes inputs, so
that the HIP library and the FP64 CPU oracle can be fed identical data.

The paper measures a 256^3 FP32 isotropic acoustic propagation with absorbing
boundaries (Section 4, Tables 2-3) but states no velocity model or source; the
generators below stand in for it (layered and smoothed-random models, Ricker
sources). Arrays are float32 with shape (nz, ny, nx), x fastest; coordinates are
float64 metres, grid point (i, j, k) at (i*hx, j*hy, k*hz).
"""
import numpy as np


def ricker(f0, dt, nt, t0=None):
    """Ricker wavelet (1 - 2 a) exp(-a), a = (pi f0 (t - t0))^2, sampled at t = n dt;
    t0 defaults to 1/f0. Returns float32 [nt]."""
    t0 = 1.0 / f0 if t0 is None else t0
    t = np.arange(nt, dtype=np.float64) * dt
    a = (np.pi * f0 * (t - t0)) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def constant(n, v):
    nx, ny, nz = n
    return np.full((nz, ny, nx), v, dtype=np.float32)


def two_layer(n, v_top=1500.0, v_bot=3000.0, k_interface=None):
    """v_top above the interface (k < k_interface), v_bot from it down."""
    nx, ny, nz = n
    k_interface = nz // 2 if k_interface is None else k_interface
    v = np.full((nz, ny, nx), v_top, dtype=np.float32)
    v[k_interface:] = v_bot
    return v


def smooth_random(n, corr_cells=20.0, seed=1):
    """Seeded white noise (PCG64) filtered with a periodic Gaussian of standard
    deviation corr_cells/sqrt(2) (so the autocorrelation std is corr_cells),
    normalised by its maximum magnitude. Returns float64 (nz, ny, nx) in [-1, 1]."""
    nx, ny, nz = n
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((nz, ny, nx))
    s = corr_cells / np.sqrt(2.0)
    kz = np.fft.fftfreq(nz)[:, None, None]
    ky = np.fft.fftfreq(ny)[None, :, None]
    kx = np.fft.rfftfreq(nx)[None, None, :]
    filt = np.exp(-2.0 * (np.pi * s) ** 2 * (kx ** 2 + ky ** 2 + kz ** 2))
    p = np.fft.irfftn(np.fft.rfftn(w) * filt, s=(nz, ny, nx), axes=(0, 1, 2))
    return p / np.max(np.abs(p))


def perturbed_two_layer(n, amp=0.05, corr_cells=20.0, seed=1, v_top=1500.0, v_bot=3000.0):
    """Two-layer model times (1 + amp * smooth_random)."""
    p = smooth_random(n, corr_cells, seed)
    return (two_layer(n, v_top, v_bot).astype(np.float64) * (1.0 + amp * p)).astype(np.float32)


def smooth_random_range(n, vmin=1500.0, vmax=4500.0, corr_cells=20.0, seed=4):
    """Smoothed random field min-max mapped onto [vmin, vmax]."""
    p = smooth_random(n, corr_cells, seed)
    p = (p - p.min()) / (p.max() - p.min())
    return (vmin + (vmax - vmin) * p).astype(np.float32)


def layered(n, nlayers, vmin=1500.0, vmax=4500.0, seed=0):
    """nlayers horizontal layers with ascending velocities drawn in [vmin, vmax]."""
    nx, ny, nz = n
    rng = np.random.Generator(np.random.PCG64(seed))
    vels = np.sort(rng.uniform(vmin, vmax, nlayers))
    cuts = np.sort(rng.choice(np.arange(1, nz), nlayers - 1, replace=False)) if nlayers > 1 else []
    v = np.empty((nz, ny, nx), dtype=np.float32)
    edges = [0] + list(cuts) + [nz]
    for L in range(nlayers):
        v[edges[L]:edges[L + 1]] = vels[L]
    return v


def gaussian_pulse(n, centre, sigma_cells):
    """exp(-|x - x_c|^2 / (2 sigma^2)) in cell units; returns float32 (nz, ny, nx)."""
    nx, ny, nz = n
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (i - centre[0]) ** 2 + (j - centre[1]) ** 2 + (k - centre[2]) ** 2
    return np.exp(-r2 / (2.0 * sigma_cells ** 2)).astype(np.float32)


def point(idx, h):
    """Metres of grid index (i, j, k), possibly fractional: float64 [1][3]."""
    return np.array([[idx[0] * h[0], idx[1] * h[1], idx[2] * h[2]]], dtype=np.float64)


def line_x(n, h, j, k):
    """Receivers at every (i, j, k), i = 0..nx-1: float64 [nx][3]."""
    nx = n[0]
    i = np.arange(nx, dtype=np.float64)
    return np.stack([i * h[0], np.full(nx, j * h[1]), np.full(nx, k * h[2])], axis=1)


def plane_z(n, h, k):
    """Receivers at every (i, j, k): float64 [ny*nx][3], x fastest."""
    nx, ny = n[0], n[1]
    jj, ii = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                         indexing="ij")
    return np.stack([ii.ravel() * h[0], jj.ravel() * h[1], np.full(nx * ny, k * h[2])], axis=1)


def random_points(n, h, count, seed, margin=0.0):
    """Uniform off-grid points inside the grid (metres), at least margin cells from
    every face."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty((count, 3))
    for a in range(3):
        out[:, a] = rng.uniform(margin, n[a] - 1 - margin, count) * h[a]
    return out


def random_field(shape, seed, dtype=np.float32):
    """Seeded standard-normal array."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape).astype(dtype)

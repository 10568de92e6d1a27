"""Shared helpers for the parity tests: case construction and error norms.

Inputs come from paper_1912_00695_amd.inputs (seeded, no solver arithmetic);
dt, the Taylor start and every expected value come from the oracle.
"""
import numpy as np

import oracle
from paper_1912_00695_amd import inputs


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = np.linalg.norm(ref)
    return np.linalg.norm(x - ref) / (n if n > 0 else 1.0)


class Case:
    """A forward problem: grid, model, sources, receivers, initial levels."""

    def __init__(self, n, h, so, nt, vel, vmax, nbl=(0,) * 6, cfl_frac=0.5, src=None,
                 wavelet=None, rec=None, u0=None, um1=None):
        self.n, self.h, self.so, self.nt = tuple(n), tuple(h), so, nt
        self.vel = np.ascontiguousarray(vel, dtype=np.float32)
        self.vmax, self.nbl = float(vmax), tuple(nbl)
        self.dt = cfl_frac * oracle.cfl_dt_max(so, vmax, h)
        self.src = np.zeros((0, 3)) if src is None else np.asarray(src, dtype=np.float64)
        self.rec = np.zeros((0, 3)) if rec is None else np.asarray(rec, dtype=np.float64)
        self.wavelet = wavelet
        self.u0, self.um1 = u0, um1

    def ogrid(self):
        return oracle.Grid(self.n, self.h, self.so, self.dt, self.nt, nbl=self.nbl,
                           vmax=self.vmax)

    def wgrid(self, storage=0, path=0, zchunk=0):
        from paper_1912_00695_amd import wave
        return wave.make_grid(self.n, self.h, self.so, self.dt, self.nt, nbl=self.nbl,
                              vmax=self.vmax, storage=storage, path=path, zchunk=zchunk)

    def oracle_forward(self):
        return oracle.forward(self.ogrid(), self.vel, self.wavelet, self.src, self.rec,
                              u0=self.u0, um1=self.um1)


def c1_case():
    """64^3, h = 10 m, SO4, v = 1500 m/s, dt = 0.5 dt_max, 100 steps, Gaussian pulse
    (sigma = 3 cells) at rest at the centre, zero Dirichlet boundary."""
    n, h = (64, 64, 64), (10.0, 10.0, 10.0)
    vel = inputs.constant(n, 1500.0)
    c = Case(n, h, 4, 100, vel, 1500.0)
    u0 = inputs.gaussian_pulse(n, (32, 32, 32), 3.0)
    c.u0 = u0
    c.um1 = oracle.taylor_start(c.ogrid(), vel, u0).astype(np.float32)
    return c


def c2_case(so, nt=500, n=(256, 256, 256)):
    """256^3, h = 10 m, two-layer 1500/3000 m/s (interface at z = n/2), 40-cell sponge,
    10 Hz Ricker at the centre, dt = 0.5 dt_max(3000), 256 receivers along x at z = 20."""
    h = (10.0, 10.0, 10.0)
    vel = inputs.two_layer(n, 1500.0, 3000.0, n[2] // 2)
    nbl = (40,) * 6 if min(n) >= 100 else (min(n) // 6,) * 6
    c = Case(n, h, so, nt, vel, 3000.0, nbl=nbl)
    c.src = inputs.point((n[0] // 2, n[1] // 2, n[2] // 2), h)
    c.wavelet = inputs.ricker(10.0, c.dt, nt)[:, None]
    c.rec = inputs.line_x(n, h, n[1] // 2, min(20, n[2] - 1))
    return c


def ragged_case(so, nt=50, n=(97, 37, 23), seed=0):
    """Several tiles with ragged edges on every axis, anisotropic spacing, variable
    velocity, asymmetric sponge, off-grid sources and receivers, random initial
    levels."""
    h = (10.0, 12.0, 9.0)
    vel = inputs.smooth_random_range(n, 1500.0, 2600.0, 6.0, seed=seed + 20)
    rng = np.random.default_rng(seed)
    c = Case(n, h, so, nt, vel, 2600.0, nbl=(5, 6, 4, 3, 2, 5))
    c.src = np.concatenate([inputs.random_points(n, h, 2, seed + 1, margin=1.0),
                            inputs.point((64, 16, 11), h)])
    c.wavelet = rng.standard_normal((nt, 3)).astype(np.float32)
    c.rec = np.concatenate([inputs.random_points(n, h, 40, seed + 2),
                            inputs.line_x(n, h, 36, 22), inputs.point((96, 0, 0), h),
                            inputs.point((64, 16, 11), h)])
    c.u0 = inputs.random_field(c.vel.shape, seed + 3) * 1e-2
    c.um1 = inputs.random_field(c.vel.shape, seed + 4) * 1e-2
    return c


def c4_case(n=(512, 512, 512), nt=1000, nbl=40, rec_stride=1):
    """SO8, smoothed-random velocity in [1500, 4500] m/s (20-cell correlation,
    seed 4), 15 Hz Ricker at the centre, dt = 0.5 dt_max(4500), receivers along x
    through the plane 10 cells below the source and at z = 20 (every rec_stride-th
    point of each line)."""
    h = (10.0, 10.0, 10.0)
    vel = inputs.smooth_random_range(n, 1500.0, 4500.0, 20.0, seed=4)
    c = Case(n, h, 8, nt, vel, 4500.0, nbl=(nbl,) * 6)
    c.src = inputs.point((n[0] // 2, n[1] // 2, n[2] // 2), h)
    c.wavelet = inputs.ricker(15.0, c.dt, nt)[:, None]
    c.rec = np.concatenate([inputs.line_x(n, h, n[1] // 2, n[2] // 2 + 10)[::rec_stride],
                            inputs.line_x(n, h, n[1] // 2, 20)[::rec_stride]])
    return c

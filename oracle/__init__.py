"""FP64 CPU oracle for the damped acoustic leapfrog scheme (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package; the HIP library never does. Two independent implementations live here:

* ``liboracle.so`` (oracle.c): the scheme stepped in plain double precision with
  OpenMP over z-planes; sizes up to the full benchmark grids.
* :mod:`oracle.brute`: dense-matrix NumPy definitions for tiny grids (the star
  Laplacian as a Kronecker sum, the time stepping as one block lower-triangular
  linear system), written from the closed-form weights with exact rationals.

The scheme (paper Section 2.1, Eq. (1); damped SO2 update of the Devito C listing in
Section 2.1; receivers and backward propagation from the conclusion's future-work
paragraph) is documented in oracle.c.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None


class OGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("hx", ctypes.c_double), ("hy", ctypes.c_double), ("hz", ctypes.c_double),
                ("so", ctypes.c_int64), ("dt", ctypes.c_double), ("nt", ctypes.c_int64),
                ("nbl", ctypes.c_int64 * 6), ("vmax", ctypes.c_double),
                ("periodic", ctypes.c_int64)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(OGrid)
        L.oracle_fd_weights.argtypes = [ctypes.c_int64, dp]
        L.oracle_fd_weights.restype = ctypes.c_int
        L.oracle_cfl_dt_max.argtypes = [ctypes.c_int64] + [ctypes.c_double] * 4
        L.oracle_cfl_dt_max.restype = ctypes.c_double
        L.oracle_sponge_1d.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                       ctypes.c_double, ctypes.c_double, dp]
        L.oracle_sponge_1d.restype = None
        L.oracle_sponge_3d.argtypes = [gp, dp]
        L.oracle_sponge_3d.restype = None
        L.oracle_laplacian.argtypes = [gp, dp, dp]
        L.oracle_laplacian.restype = ctypes.c_int
        L.oracle_trilinear.argtypes = [gp, dp, ctypes.POINTER(ctypes.c_int64), dp]
        L.oracle_trilinear.restype = ctypes.c_int
        L.oracle_forward.argtypes = [gp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                     dp, dp, dp, dp]
        L.oracle_forward.restype = ctypes.c_int
        L.oracle_adjoint.argtypes = [gp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp, dp]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_gradient.argtypes = [gp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                      ctypes.c_int64, dp, dp, dp]
        L.oracle_gradient.restype = ctypes.c_int
        L.oracle_gradient_image.argtypes = [gp, dp, dp, dp, ctypes.c_int, dp, ctypes.c_int, dp,
                                            ctypes.c_int64, dp, dp, dp, dp]
        L.oracle_gradient_image.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_set_num_threads.restype = None
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _d(a, shape=None):
    """Contiguous float64 copy (or None)."""
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class Grid:
    """Grid description: n = (nx, ny, nz), h = (hx, hy, hz) metres, even space order
    so, time step dt seconds, nt steps, sponge widths nbl (x-,x+,y-,y+,z-,z+), sponge
    reference velocity vmax m/s, periodic halo flag (oracle-only test mode)."""

    def __init__(self, n, h, so, dt, nt, nbl=(0,) * 6, vmax=1500.0, periodic=False):
        self.n = tuple(int(v) for v in n)
        self.h = tuple(float(v) for v in h)
        self.so, self.dt, self.nt = int(so), float(dt), int(nt)
        self.nbl = tuple(int(v) for v in nbl)
        self.vmax, self.periodic = float(vmax), bool(periodic)

    @property
    def shape(self):
        """Array shape (nz, ny, nx), x fastest."""
        return (self.n[2], self.n[1], self.n[0])

    @property
    def npts(self):
        return self.n[0] * self.n[1] * self.n[2]

    def c(self):
        g = OGrid()
        g.nx, g.ny, g.nz = self.n
        g.hx, g.hy, g.hz = self.h
        g.so, g.dt, g.nt = self.so, self.dt, self.nt
        for i, v in enumerate(self.nbl):
            g.nbl[i] = v
        g.vmax, g.periodic = self.vmax, int(self.periodic)
        return g

    def replace(self, **kw):
        d = dict(n=self.n, h=self.h, so=self.so, dt=self.dt, nt=self.nt, nbl=self.nbl,
                 vmax=self.vmax, periodic=self.periodic)
        d.update(kw)
        return Grid(**d)


def fd_weights(so):
    """Second-derivative weights w[0..r] by Fornberg's recursion."""
    w = np.zeros(so // 2 + 1)
    if lib().oracle_fd_weights(so, _p(w)) != 0:
        raise ValueError("bad space order %r" % (so,))
    return w


def cfl_dt_max(so, vmax, h):
    hx, hy, hz = h
    return lib().oracle_cfl_dt_max(so, vmax, hx, hy, hz)


def sponge_1d(n, lo, hi, h, vmax):
    g = np.zeros(n)
    lib().oracle_sponge_1d(n, lo, hi, h, vmax, _p(g))
    return g


def sponge_3d(grid):
    g = np.zeros(grid.shape)
    lib().oracle_sponge_3d(ctypes.byref(grid.c()), _p(g))
    return g


def laplacian(grid, u):
    u = _d(u, grid.shape)
    out = np.zeros(grid.shape)
    if lib().oracle_laplacian(ctypes.byref(grid.c()), _p(u), _p(out)) != 0:
        raise ValueError("bad grid")
    return out


def trilinear(grid, xyz):
    """Corners of a point (metres): (flat indices, weights)."""
    x = _d(xyz, (3,))
    idx = np.zeros(8, dtype=np.int64)
    w = np.zeros(8)
    c = lib().oracle_trilinear(ctypes.byref(grid.c()), _p(x),
                               idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _p(w))
    if c < 0:
        raise ValueError("point outside the grid")
    return idx[:c].copy(), w[:c].copy()


def taylor_start(grid, vel, u0):
    """u^{-1} = u0 + dt^2 v^2 L_h u0 / 2: the second-order start for a field at rest
    (zero initial velocity), so that u^1 = u^{-1} when there is no damping."""
    vel = _d(vel, grid.shape)
    u0 = _d(u0, grid.shape)
    return u0 + 0.5 * grid.dt ** 2 * vel ** 2 * laplacian(grid, u0)


def forward(grid, vel, wavelet=None, src_xyz=None, rec_xyz=None, u0=None, um1=None):
    """Forward solve. Returns (rec [nt][nrec], u^{nt}, u^{nt-1})."""
    vel = _d(vel, grid.shape)
    src = _d(src_xyz if src_xyz is not None else np.zeros((0, 3))).reshape(-1, 3)
    rec = _d(rec_xyz if rec_xyz is not None else np.zeros((0, 3))).reshape(-1, 3)
    ns, nr = src.shape[0], rec.shape[0]
    wav = _d(wavelet if wavelet is not None else np.zeros((grid.nt, 0))).reshape(grid.nt, ns)
    out = np.zeros((grid.nt, nr))
    uf = np.zeros(grid.shape)
    umf = np.zeros(grid.shape)
    rc = lib().oracle_forward(ctypes.byref(grid.c()), _p(vel), _p(wav), _p(src), ns, _p(rec), nr,
                              _p(out), _p(_d(u0, grid.shape)), _p(_d(um1, grid.shape)),
                              _p(uf), _p(umf))
    if rc != 0:
        raise ValueError("oracle_forward failed (%d)" % rc)
    return out, uf, umf


def adjoint(grid, vel, rec_data, rec_xyz, src_xyz):
    """Adjoint solve. Returns (src_out [nt][nsrc], lambda^0)."""
    vel = _d(vel, grid.shape)
    rec = _d(rec_xyz).reshape(-1, 3)
    src = _d(src_xyz).reshape(-1, 3)
    nr, ns = rec.shape[0], src.shape[0]
    d = _d(rec_data).reshape(grid.nt, nr)
    out = np.zeros((grid.nt, ns))
    lam = np.zeros(grid.shape)
    rc = lib().oracle_adjoint(ctypes.byref(grid.c()), _p(vel), _p(d), _p(rec), nr, _p(src), ns,
                              _p(out), _p(lam))
    if rc != 0:
        raise ValueError("oracle_adjoint failed (%d)" % rc)
    return out, lam


def gradient(grid, vel, wavelet, src_xyz, rec_xyz, rec_grad, ckpt_every=0):
    """Gradient for dL/dd = rec_grad. Returns (grad_m, grad_vel, grad_wavelet)."""
    vel = _d(vel, grid.shape)
    src = _d(src_xyz).reshape(-1, 3)
    rec = _d(rec_xyz).reshape(-1, 3)
    ns, nr = src.shape[0], rec.shape[0]
    wav = _d(wavelet).reshape(grid.nt, ns)
    rg = _d(rec_grad).reshape(grid.nt, nr)
    gm = np.zeros(grid.shape)
    gv = np.zeros(grid.shape)
    gw = np.zeros((grid.nt, ns))
    rc = lib().oracle_gradient(ctypes.byref(grid.c()), _p(vel), _p(wav), _p(src), ns, _p(rec), nr,
                               _p(rg), int(ckpt_every), _p(gm), _p(gv), _p(gw))
    if rc != 0:
        raise ValueError("oracle_gradient failed (%d)" % rc)
    return gm, gv, gw


def rtm_image(grid, vel, wavelet, src_xyz, rec_xyz, rec_data, ckpt_every=0):
    """Zero-lag cross-correlation image sum_{n=1..nt} u^n lambda^n of the forward field
    (sources) with the adjoint field driven by rec_data at the receivers."""
    vel = _d(vel, grid.shape)
    src = _d(src_xyz).reshape(-1, 3)
    rec = _d(rec_xyz).reshape(-1, 3)
    ns, nr = src.shape[0], rec.shape[0]
    wav = _d(wavelet).reshape(grid.nt, ns)
    rd = _d(rec_data).reshape(grid.nt, nr)
    img = np.zeros(grid.shape)
    rc = lib().oracle_gradient_image(ctypes.byref(grid.c()), _p(vel), _p(wav), _p(src), ns,
                                     _p(rec), nr, _p(rd), int(ckpt_every), None, None, None,
                                     _p(img))
    if rc != 0:
        raise ValueError("oracle_gradient_image failed (%d)" % rc)
    return img


def num_threads():
    return lib().oracle_num_threads()


def set_num_threads(n):
    """Threads of the following oracle calls (timing only; results do not depend on
    it: every loop writes disjoint points)."""
    lib().oracle_set_num_threads(int(n))

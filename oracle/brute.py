"""Dense-matrix brute force for tiny grids (test infrastructure).

Independent of oracle.c: nothing here calls the C library. Every object is built
from its definition:

* weights from the closed form of the centred second-derivative stencil, in exact
  rationals: w_q = 2 (-1)^{q+1} (r!)^2 / (q^2 (r-q)! (r+q)!), w_0 = -2 sum_q 1/q^2;
* the star Laplacian as the Kronecker sum of three 1D matrices (zero or periodic
  halo);
* the time stepping not as an update formula but as the discrete PDE
  m (u^{n+1} - 2u^n + u^{n-1}) / dt^2 + m gamma (u^{n+1} - u^{n-1}) / (2 dt) - L_h u^n
      = P^T s^n       (paper Eq. (1) with the damping term of its damped SO2 listing)
  for n = 0..nt-1, assembled into one block lower-triangular system and solved
  with a dense LU solve;
* the forward map F: s -> d as an explicit matrix, its transpose giving the
  adjoint.
"""
from fractions import Fraction
from math import factorial, floor, log, pi, sin

import numpy as np


def weights_exact(so):
    """Closed-form second-derivative weights as Fractions w[0..r]."""
    r = so // 2
    w = [Fraction(0)] * (r + 1)
    for q in range(1, r + 1):
        w[q] = Fraction(2 * (-1) ** (q + 1) * factorial(r) ** 2,
                        q * q * factorial(r - q) * factorial(r + q))
    w[0] = -2 * sum(Fraction(1, q * q) for q in range(1, r + 1))
    return w


def d2_matrix(n, h, so, periodic=False):
    """1D second-derivative matrix of order so on n points, spacing h."""
    w = [float(x) for x in weights_exact(so)]
    r = so // 2
    D = np.zeros((n, n))
    for i in range(n):
        for q in range(-r, r + 1):
            j = i + q
            if periodic:
                D[i, j % n] += w[abs(q)]
            elif 0 <= j < n:
                D[i, j] += w[abs(q)]
    return D / (h * h)


def lap_matrix(n, h, so, periodic=False):
    """Star Laplacian on an nx*ny*nz grid, flat index (k*ny + j)*nx + i."""
    nx, ny, nz = n
    hx, hy, hz = h
    Ix, Iy, Iz = np.eye(nx), np.eye(ny), np.eye(nz)
    return (np.kron(np.kron(Iz, Iy), d2_matrix(nx, hx, so, periodic))
            + np.kron(np.kron(Iz, d2_matrix(ny, hy, so, periodic)), Ix)
            + np.kron(np.kron(d2_matrix(nz, hz, so, periodic), Iy), Ix))


def sponge_profile(n, lo, hi, h, vmax, R=1e-3):
    """Sponge gamma along one axis (1/s): gmax (p - sin(2 pi p)/(2 pi)),
    p = (nbl - d)/nbl at distance index d from a face, gmax = 3 vmax ln(1/R)/(2 nbl h)."""
    g = np.zeros(n)
    for face, nbl in ((0, lo), (1, hi)):
        if nbl <= 0:
            continue
        gmax = 1.5 * vmax * log(1.0 / R) / (nbl * h)
        for d in range(min(nbl, n)):
            p = (nbl - d) / nbl
            i = d if face == 0 else n - 1 - d
            g[i] += gmax * (p - sin(2 * pi * p) / (2 * pi))
    return g


def gamma_field(n, h, nbl, vmax):
    nx, ny, nz = n
    gx = sponge_profile(nx, nbl[0], nbl[1], h[0], vmax)
    gy = sponge_profile(ny, nbl[2], nbl[3], h[1], vmax)
    gz = sponge_profile(nz, nbl[4], nbl[5], h[2], vmax)
    return (gz[:, None, None] + gy[None, :, None] + gx[None, None, :]).ravel()


def interp_matrix(n, h, xyz):
    """Trilinear interpolation rows (npts x N) for points given in metres."""
    nx, ny, nz = n
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    M = np.zeros((xyz.shape[0], nx * ny * nz))
    for s, (x, y, z) in enumerate(xyz):
        f = [x / h[0], y / h[1], z / h[2]]
        base, frac = [], []
        for a, nn in enumerate((nx, ny, nz)):
            if not (0.0 <= f[a] <= nn - 1):
                raise ValueError("point outside the grid")
            b = int(floor(f[a]))
            base.append(b)
            frac.append(f[a] - b)
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = ((frac[0] if dx else 1 - frac[0]) * (frac[1] if dy else 1 - frac[1])
                         * (frac[2] if dz else 1 - frac[2]))
                    if w == 0.0:
                        continue
                    i, j, k = base[0] + dx, base[1] + dy, base[2] + dz
                    M[s, (k * ny + j) * nx + i] += w
    return M


def system(n, h, so, dt, nt, vel, nbl=(0,) * 6, vmax=1500.0, periodic=False):
    """Block lower-triangular matrix of the discrete PDE for the unknowns
    U = (u^1, ..., u^nt), and the blocks (A_next, A_cur, A_prev) of one row."""
    N = n[0] * n[1] * n[2]
    m = 1.0 / np.asarray(vel, dtype=np.float64).ravel() ** 2
    gam = gamma_field(n, h, nbl, vmax)
    L = lap_matrix(n, h, so, periodic)
    A_next = np.diag(m / dt ** 2 + m * gam / (2 * dt))
    A_cur = -np.diag(2 * m / dt ** 2) - L
    A_prev = np.diag(m / dt ** 2 - m * gam / (2 * dt))
    T = np.zeros((nt * N, nt * N))
    for row in range(nt):  # equation n = row produces u^{row+1}
        T[row * N:(row + 1) * N, row * N:(row + 1) * N] = A_next
        if row >= 1:
            T[row * N:(row + 1) * N, (row - 1) * N:row * N] = A_cur
        if row >= 2:
            T[row * N:(row + 1) * N, (row - 2) * N:(row - 1) * N] = A_prev
    return T, (A_next, A_cur, A_prev)


def forward(n, h, so, dt, nt, vel, wavelet=None, src_xyz=None, rec_xyz=None, u0=None, um1=None,
            nbl=(0,) * 6, vmax=1500.0, periodic=False):
    """Solve the whole space-time system at once. Returns (rec [nt][nrec], U [nt][N])
    where U[n] = u^{n+1}."""
    N = n[0] * n[1] * n[2]
    T, (A_next, A_cur, A_prev) = system(n, h, so, dt, nt, vel, nbl, vmax, periodic)
    rhs = np.zeros((nt, N))
    if src_xyz is not None and len(src_xyz):
        P = interp_matrix(n, h, src_xyz)
        rhs += np.asarray(wavelet, dtype=np.float64).reshape(nt, -1) @ P
    u0 = np.zeros(N) if u0 is None else np.asarray(u0, dtype=np.float64).ravel()
    um1 = np.zeros(N) if um1 is None else np.asarray(um1, dtype=np.float64).ravel()
    if nt >= 1:
        rhs[0] -= A_cur @ u0 + A_prev @ um1
    if nt >= 2:
        rhs[1] -= A_prev @ u0
    U = np.linalg.solve(T, rhs.ravel()).reshape(nt, N)
    if rec_xyz is not None and len(rec_xyz):
        R = interp_matrix(n, h, rec_xyz)
        rec = U @ R.T
    else:
        rec = np.zeros((nt, 0))
    return rec, U


def forward_matrix(n, h, so, dt, nt, vel, src_xyz, rec_xyz, nbl=(0,) * 6, vmax=1500.0):
    """Dense F with rec.ravel() = F @ wavelet.ravel() (zero initial state)."""
    N = n[0] * n[1] * n[2]
    T, _ = system(n, h, so, dt, nt, vel, nbl, vmax)
    P = interp_matrix(n, h, src_xyz)
    R = interp_matrix(n, h, rec_xyz)
    Tinv = np.linalg.inv(T)
    Pbig = np.kron(np.eye(nt), P.T)      # (nt N) x (nt nsrc)
    Rbig = np.kron(np.eye(nt), R)        # (nt nrec) x (nt N)
    del N
    return Rbig @ Tinv @ Pbig


def adjoint_levels(n, h, so, dt, nt, vel, rec_xyz, rec_data, nbl=(0,) * 6, vmax=1500.0):
    """Adjoint levels lambda^0..lambda^{nt-1} from the transposed space-time system of
    the discrete PDE: T^T mu = (I (x) R^T) d, where row n of T is the equation that
    produces u^{n+1} and receives P^T s^n, so F^T d = (I (x) P) mu and lambda^n = mu_n.
    Returns [nt][N]."""
    N = n[0] * n[1] * n[2]
    T, _ = system(n, h, so, dt, nt, vel, nbl, vmax)
    R = interp_matrix(n, h, rec_xyz)
    rhs = (np.asarray(rec_data, dtype=np.float64).reshape(nt, -1) @ R).ravel()
    return np.linalg.solve(T.T, rhs).reshape(nt, N)

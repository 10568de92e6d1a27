"""Pins of the oracle's Laplacian, sponge and trilinear operators."""
import numpy as np
import pytest

import oracle
from oracle import brute


@pytest.mark.parametrize("so", [2, 4, 6, 8])
@pytest.mark.parametrize("periodic", [False, True])
def test_laplacian_matches_dense_kronecker_sum(so, periodic):
    n, h = (7, 6, 5), (10.0, 7.0, 13.0)
    if periodic and so > 4:
        n = (11, 10, 9)  # periodic wrap needs n > 2r to keep the stencil distinct
    g = oracle.Grid(n, h, so, 1e-3, 1, periodic=periodic)
    u = np.random.default_rng(so).standard_normal(g.shape)
    L = brute.lap_matrix(n, h, so, periodic)
    np.testing.assert_allclose(oracle.laplacian(g, u).ravel(), L @ u.ravel(), rtol=1e-12,
                               atol=1e-12 * np.abs(L).max() * np.abs(u).max())


def test_dense_laplacian_symmetric():
    for so in (2, 4, 8):
        L = brute.lap_matrix((7, 6, 5), (10.0, 7.0, 13.0), so)
        np.testing.assert_allclose(L, L.T, rtol=0, atol=1e-15)


@pytest.mark.parametrize("so", [2, 4, 8, 12])
def test_laplacian_self_adjoint(so):
    g = oracle.Grid((20, 17, 15), (10.0, 8.0, 12.0), so, 1e-3, 1)
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal(g.shape), rng.standard_normal(g.shape)
    lab = np.vdot(oracle.laplacian(g, a), b)
    alb = np.vdot(a, oracle.laplacian(g, b))
    assert abs(lab - alb) <= 1e-12 * abs(lab)


@pytest.mark.parametrize("so", [2, 4, 6, 8])
def test_laplacian_exact_on_polynomials(so):
    # Away from the halo the order-SO stencil differentiates polynomials of degree
    # <= SO+1 exactly (per axis); the analytic Laplacian of x^a y^b z^c is known.
    r = so // 2
    n = (2 * r + 5, 2 * r + 4, 2 * r + 3)
    h = (0.5, 0.25, 0.4)
    g = oracle.Grid(n, h, so, 1e-3, 1)
    k, j, i = np.meshgrid(*(np.arange(nn, dtype=np.float64) for nn in g.shape), indexing="ij")
    x, y, z = (i - n[0] / 2) * h[0], (j - n[1] / 2) * h[1], (k - n[2] / 2) * h[2]
    deg = so + 1
    for (a, b, c) in [(deg, 0, 0), (0, deg, 0), (0, 0, deg), (2, so, 1), (so - 1, 2, 3)]:
        u = x ** a * y ** b * z ** c
        lap = (a * (a - 1) * x ** max(a - 2, 0) * y ** b * z ** c if a >= 2 else 0 * x) \
            + (b * (b - 1) * x ** a * y ** max(b - 2, 0) * z ** c if b >= 2 else 0 * x) \
            + (c * (c - 1) * x ** a * y ** b * z ** max(c - 2, 0) if c >= 2 else 0 * x)
        got = oracle.laplacian(g, u)
        sl = (slice(r, n[2] - r), slice(r, n[1] - r), slice(r, n[0] - r))
        scale = np.abs(u[sl]).max() / min(h) ** 2 + 1.0
        np.testing.assert_allclose(got[sl], lap[sl], rtol=0, atol=1e-9 * scale)


def test_sponge_profile_shape():
    n, nbl, h, v = 100, 20, 10.0, 3000.0
    g = oracle.sponge_1d(n, nbl, nbl, h, v)
    gmax = 1.5 * v * np.log(1e3) / (nbl * h)
    assert g[0] == pytest.approx(gmax, rel=1e-14) and g[-1] == pytest.approx(gmax, rel=1e-14)
    assert np.all(g[nbl:n - nbl] == 0.0)
    assert np.all(np.diff(g[:nbl]) < 0) and np.all(np.diff(g[n - nbl:]) > 0)
    np.testing.assert_allclose(g, brute.sponge_profile(n, nbl, nbl, h, v), rtol=1e-14, atol=0)
    # per-face widths, asymmetric, and the 3D field is the sum of the three axes
    grid = oracle.Grid((12, 10, 9), (10.0, 5.0, 20.0), 4, 1e-3, 1, nbl=(3, 0, 2, 4, 0, 5), vmax=v)
    np.testing.assert_allclose(oracle.sponge_3d(grid).ravel(),
                               brute.gamma_field(grid.n, grid.h, grid.nbl, v), rtol=1e-14, atol=0)


def test_trilinear_exact_on_linear_fields():
    g = oracle.Grid((9, 8, 7), (10.0, 5.0, 20.0), 4, 1e-3, 1)
    k, j, i = np.meshgrid(*(np.arange(nn, dtype=np.float64) for nn in g.shape), indexing="ij")
    f = 3.0 + 0.7 * i * g.h[0] - 1.3 * j * g.h[1] + 0.2 * k * g.h[2]
    rng = np.random.default_rng(3)
    pts = np.concatenate([rng.uniform(0, 1, (50, 3)) * (np.array(g.n) - 1) * np.array(g.h),
                          np.array([[0.0, 0.0, 0.0], [80.0, 35.0, 120.0], [40.0, 20.0, 60.0]])])
    for p in pts:
        idx, w = oracle.trilinear(g, p)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert np.dot(w, f.ravel()[idx]) == pytest.approx(3.0 + 0.7 * p[0] - 1.3 * p[1] + 0.2 * p[2],
                                                          rel=1e-13)
    idx, w = oracle.trilinear(g, [40.0, 20.0, 60.0])  # on-grid: one corner of weight 1
    assert len(idx) == 1 and w[0] == 1.0 and idx[0] == (3 * 8 + 4) * 9 + 4
    with pytest.raises(ValueError):
        oracle.trilinear(g, [81.0, 0.0, 0.0])

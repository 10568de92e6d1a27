"""Pins of the oracle's adjoint and gradient."""
import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1912_00695_amd import inputs


def _setup(n=(14, 12, 11), so=4, nt=40, nbl=(3,) * 6, seed=0):
    h = (10.0, 9.0, 11.0)
    vel = inputs.smooth_random_range(n, 1500.0, 2500.0, 3.0, seed=seed).astype(np.float64)
    dt = 0.5 * oracle.cfl_dt_max(so, 2500.0, h)
    g = oracle.Grid(n, h, so, dt, nt, nbl=nbl, vmax=2500.0)
    src = np.array([[61.7, 48.2, 51.3], [30.0, 27.0, 44.0]])
    rec = np.concatenate([inputs.line_x(n, h, 4, 2), [[77.7, 20.1, 90.9]]])
    return g, vel, src, rec


@pytest.mark.parametrize("so", [2, 4, 8])
def test_dot_product(so):
    g, vel, src, rec = _setup(so=so)
    rng = np.random.default_rng(2)
    s = rng.standard_normal((g.nt, len(src)))
    d = rng.standard_normal((g.nt, len(rec)))
    Fs = oracle.forward(g, vel, s, src, rec)[0]
    Ftd = oracle.adjoint(g, vel, d, rec, src)[0]
    a, b = np.vdot(Fs, d), np.vdot(s, Ftd)
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_adjoint_matches_dense_transpose():
    n, h, so, nt = (5, 4, 4), (10.0, 12.0, 9.0), 4, 7
    rng = np.random.default_rng(5)
    vel = rng.uniform(1500, 2500, n[::-1])
    dt = 0.5 * oracle.cfl_dt_max(so, 2500.0, h)
    nbl = (1, 2, 0, 1, 1, 0)
    g = oracle.Grid(n, h, so, dt, nt, nbl=nbl, vmax=2500.0)
    src = np.array([[13.3, 17.9, 9.4]])
    rec = np.array([[5.5, 30.0, 27.0], [30.0, 12.0, 13.5]])
    F = brute.forward_matrix(n, h, so, dt, nt, vel, src, rec, nbl=nbl, vmax=2500.0)
    d = rng.standard_normal((nt, 2))
    want = (F.T @ d.ravel()).reshape(nt, 1)
    got = oracle.adjoint(g, vel, d, rec, src)[0]
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    s = rng.standard_normal((nt, 1))
    np.testing.assert_allclose(oracle.forward(g, vel, s, src, rec)[0].ravel(), F @ s.ravel(),
                               rtol=1e-9, atol=1e-9 * np.abs(F @ s.ravel()).max())


def test_reciprocity():
    """Swapping an on-grid source and receiver leaves the trace unchanged (the
    space-time operator has symmetric blocks, variable velocity and sponge
    included)."""
    g, vel, _, _ = _setup(nt=60)
    A = np.array([[30.0, 36.0, 22.0]])
    B = np.array([[100.0, 72.0, 88.0]])
    w = inputs.ricker(15.0, g.dt, g.nt).astype(np.float64)[:, None]
    ab = oracle.forward(g, vel, w, A, B)[0]
    ba = oracle.forward(g, vel, w, B, A)[0]
    assert np.abs(ab).max() > 0
    np.testing.assert_allclose(ab, ba, rtol=0, atol=1e-12 * np.abs(ab).max())


def _misfit(g, vel, w, src, rec, obs):
    d = oracle.forward(g, vel, w, src, rec)[0]
    return 0.5 * np.sum((d - obs) ** 2), d


def test_gradient_taylor():
    """J(m + e dm) - J(m) - e <g, dm> = O(e^2)."""
    g, vel, src, rec = _setup(nt=50)
    w = np.tile(inputs.ricker(12.0, g.dt, g.nt).astype(np.float64)[:, None], (1, 2))
    vtrue = vel * (1 + 0.03 * inputs.smooth_random(g.n, 3.0, seed=9))
    obs = oracle.forward(g, vtrue, w, src, rec)[0]
    J0, d0 = _misfit(g, vel, w, src, rec, obs)
    gm, gv, _ = oracle.gradient(g, vel, w, src, rec, d0 - obs)
    m = 1.0 / vel ** 2
    dm = m * 0.1 * inputs.smooth_random(g.n, 3.0, seed=10)
    res = []
    for e in (1e-1, 5e-2, 2.5e-2, 1.25e-2):
        J1 = _misfit(g, 1.0 / np.sqrt(m + e * dm), w, src, rec, obs)[0]
        res.append(abs(J1 - J0 - e * np.vdot(gm, dm)))
    ratios = [a / b for a, b in zip(res, res[1:])]
    assert all(3.5 < r < 4.5 for r in ratios), ratios
    # chain rule to velocity
    np.testing.assert_allclose(gv, -2.0 * gm / vel ** 3, rtol=1e-14)


def test_gradient_matches_brute_force_fd():
    """Central differences of J through the dense space-time solve, point by point."""
    n, h, so, nt = (5, 4, 3), (10.0, 10.0, 10.0), 2, 8
    rng = np.random.default_rng(8)
    vel = rng.uniform(1500, 2000, n[::-1])
    dt = 0.5 * oracle.cfl_dt_max(so, 2100.0, h)
    nbl = (1, 1, 0, 1, 1, 0)
    g = oracle.Grid(n, h, so, dt, nt, nbl=nbl, vmax=2100.0)
    src = np.array([[21.0, 14.0, 10.0]])
    rec = np.array([[5.0, 22.0, 17.0], [35.0, 30.0, 0.0]])
    w = rng.standard_normal((nt, 1))
    obs = rng.standard_normal((nt, 2)) * 1e-3
    d0 = oracle.forward(g, vel, w, src, rec)[0]
    gm, _, gw = oracle.gradient(g, vel, w, src, rec, d0 - obs)
    m = (1.0 / vel ** 2).ravel()

    def J(mm):
        d = brute.forward(n, h, so, dt, nt, 1.0 / np.sqrt(mm.reshape(vel.shape)), w, src, rec,
                          nbl=nbl, vmax=2100.0)[0]
        return 0.5 * np.sum((d - obs) ** 2)

    fd = np.zeros_like(m)
    for p in range(m.size):
        e = 1e-4 * m[p]
        mp, mm_ = m.copy(), m.copy()
        mp[p] += e
        mm_[p] -= e
        fd[p] = (J(mp) - J(mm_)) / (2 * e)
    np.testing.assert_allclose(gm.ravel(), fd, rtol=1e-5, atol=1e-6 * np.abs(fd).max())
    # wavelet gradient = F^T r
    F = brute.forward_matrix(n, h, so, dt, nt, vel, src, rec, nbl=nbl, vmax=2100.0)
    np.testing.assert_allclose(gw.ravel(), F.T @ (d0 - obs).ravel(), rtol=1e-8,
                               atol=1e-10 * np.abs(gw).max())


def test_checkpoint_schedule_is_exact():
    g, vel, src, rec = _setup(nt=23)
    rng = np.random.default_rng(4)
    w = rng.standard_normal((g.nt, 2))
    r = rng.standard_normal((g.nt, len(rec)))
    full = oracle.gradient(g, vel, w, src, rec, r, ckpt_every=0)
    for C in (1, 5, 7, 22, 23):
        part = oracle.gradient(g, vel, w, src, rec, r, ckpt_every=C)
        for a, b in zip(full, part):
            np.testing.assert_array_equal(a, b)


def test_rtm_image_matches_dense_levels():
    """Image = sum_n u^n lambda^n with u^n from the dense forward solve and lambda^n
    from the dense transposed system (lambda^{nt} = 0)."""
    n, h, so, nt = (5, 4, 4), (10.0, 12.0, 9.0), 4, 8
    rng = np.random.default_rng(21)
    vel = rng.uniform(1500, 2500, n[::-1])
    dt = 0.5 * oracle.cfl_dt_max(so, 2500.0, h)
    nbl = (1, 1, 0, 1, 1, 0)
    g = oracle.Grid(n, h, so, dt, nt, nbl=nbl, vmax=2500.0)
    src = np.array([[13.3, 17.9, 9.4]])
    rec = np.array([[5.5, 30.0, 27.0], [30.0, 12.0, 13.5]])
    w = rng.standard_normal((nt, 1))
    d = rng.standard_normal((nt, 2))
    _, U = brute.forward(n, h, so, dt, nt, vel, w, src, rec, nbl=nbl, vmax=2500.0)
    lam = brute.adjoint_levels(n, h, so, dt, nt, vel, rec, d, nbl=nbl, vmax=2500.0)
    # U[j-1] = u^j (j = 1..nt), lam[j] = lambda^j (j = 0..nt-1), lambda^nt = 0
    want = sum(U[j - 1] * lam[j] for j in range(1, nt))
    for C in (0, 3):
        got = oracle.rtm_image(g, vel, w, src, rec, d, ckpt_every=C).ravel()
        np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-9 * np.abs(want).max())
    # the adjoint levels themselves agree with the stepping adjoint's sampled output
    src_o, lam0 = oracle.adjoint(g, vel, d, rec, src)
    np.testing.assert_allclose(lam0.ravel(), lam[0], rtol=1e-9, atol=1e-9 * np.abs(lam[0]).max())

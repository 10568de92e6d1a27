"""Pins of the oracle's finite-difference weights and stability limit.

The weights come from Fornberg's recursion in oracle.c; they are pinned to the
closed form of the centred second-derivative stencil (exact rationals), to the
moment conditions that define that stencil, and to the SO2 stencil printed in
the paper's damped update listing (Section 2.1). The stability limit is pinned to
a direct numerical maximisation of the discrete symbol.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("so", list(range(2, 26, 2)))
def test_fornberg_matches_closed_form(so):
    w = oracle.fd_weights(so)
    ex = [float(x) for x in brute.weights_exact(so)]
    np.testing.assert_allclose(w, ex, rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("so", list(range(2, 26, 2)))
def test_closed_form_moments_exact(so):
    # sum_{q=-r..r} w_q q^(2j) = 0 (j = 0), 2 (j = 1), 0 (j = 2..r): exact rationals.
    w = brute.weights_exact(so)
    r = so // 2
    for j in range(0, r + 1):
        s = w[0] * (1 if j == 0 else 0) + 2 * sum(w[q] * Fraction(q) ** (2 * j) for q in range(1, r + 1))
        assert s == (2 if j == 1 else 0), (so, j, s)


@pytest.mark.parametrize("so", list(range(2, 26, 2)))
def test_fornberg_moments_numeric(so):
    w = oracle.fd_weights(so)
    r = so // 2
    q = np.arange(1, r + 1, dtype=np.float64)
    for j in range(0, r + 1):
        s = (w[0] if j == 0 else 0.0) + 2.0 * np.sum(w[1:] * q ** (2 * j))
        scale = 2.0 * np.sum(np.abs(w[1:]) * q ** (2 * j)) + abs(w[0])
        assert abs(s - (2.0 if j == 1 else 0.0)) <= 1e-12 * scale


def test_so2_weights_match_paper_listing():
    # The paper's SO2 update at unit spacing weighs the six face neighbours by 1 and
    # the centre by -6 (the fixture states those two values with their citation):
    # per axis w1 = 1 and w0 = -2.
    fx = json.load(open(os.path.join(GOLDEN, "so2_stencil.json")))
    w = oracle.fd_weights(2)
    assert w[1] == fx["face_neighbour_weight"]
    assert 3 * w[0] == fx["centre_weight"]


@pytest.mark.parametrize("so", [2, 4, 8, 12, 16, 24])
@pytest.mark.parametrize("h", [(10.0, 10.0, 10.0), (5.0, 10.0, 20.0)])
def test_cfl_matches_symbol_maximum(so, h):
    # dt_max = 2 / (v sqrt(max_k symbol)), the symbol sum_a h_a^-2 (-w0 - 2 sum_q w_q cos(q k h_a))
    # maximised numerically over a fine wavenumber grid with exact-rational weights.
    w = [float(x) for x in brute.weights_exact(so)]
    th = np.linspace(0.0, np.pi, 20001)
    sym1 = -w[0] - 2.0 * sum(w[q] * np.cos(q * th) for q in range(1, so // 2 + 1))
    lam = sum(sym1.max() / ha ** 2 for ha in h)
    v = 3000.0
    expect = 2.0 / (v * np.sqrt(lam))
    assert oracle.cfl_dt_max(so, v, h) == pytest.approx(expect, rel=1e-12)


@pytest.mark.parametrize("so", [2, 4, 8])
def test_cfl_stability_boundary(so):
    # Periodic 8^3 grid holds the Nyquist mode exactly: just below the limit the
    # solution stays bounded, just above it grows exponentially.
    h = (10.0, 10.0, 10.0)
    v = 2000.0
    dtm = oracle.cfl_dt_max(so, v, h)
    u0 = np.random.default_rng(0).standard_normal((8, 8, 8))
    vel = np.full((8, 8, 8), v)
    for fac, grows in ((0.99, False), (1.05, True)):
        g = oracle.Grid((8, 8, 8), h, so, fac * dtm, 400, periodic=True, vmax=v)
        _, uf, _ = oracle.forward(g, vel, u0=u0, um1=u0)
        growth = np.max(np.abs(uf)) / np.max(np.abs(u0))
        if grows:
            assert growth > 1e6
        else:
            assert growth < 1e3

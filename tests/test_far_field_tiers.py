"""Distance tiers of the mixed path's far field, checked on the host (no GPU).

A line whose window covers a 1024-point tile, whose |x| < 15 zone misses it
and whose centre lies more than 64 points outside it adds a smooth function
to the tile.  The nearer such lines (centre 65 to 128 points away) are
evaluated at 16 Chebyshev points in each 256-point quarter, one line per
64-lane pass; the farther ones at fewer Chebyshev points of the whole tile,
so that one pass takes several lines:
    centre beyond 128 points: 32 nodes, 2 lines per pass
    beyond 384:               16 nodes, 4 lines per pass
    beyond 1536:               8 nodes, 8 lines per pass
At the end of the tile each whole-tile interpolant is evaluated at the 64
quarter nodes (a fixed 64 x 56 matrix of Lagrange basis values, rounded to
FP32) and added to the quarter nodes' sums, which are then interpolated
per quarter as before.

This test runs that chain in FP32 arithmetic (numpy float32, node values
rounded from float64) for one line at the nearest centre each tier allows,
and compares with the line's two-node fraction in float64 at every point of
the tile: damping 1e-4 to 1e5 (both branches of the fraction), Doppler
widths of 1 to 100 grid points, centres on either side.  Each tier stays
within 2.5e-6 of the line's part, below the 1.5e-5 bound of the per-quarter
rule at its own edge and far below the fraction's own 5e-5 at |x| = 15; a
centre inside a tier's band breaks its bound, so the cases do probe the
edges.
"""
import math

import numpy as np
import pytest

LNQ = math.log1p(1.0 / 5e5)
TILE = 1024
QUARTER = 256
F32 = np.float32
# (nodes over the whole tile, nearest allowed centre distance in points)
TIERS = [(32, 128), (16, 384), (8, 1536)]
BOUND = 2.5e-6


def fraction(j, jstar, a, b):
    """Two-node Gauss-Hermite pair of S H (S = 1) at fine index j, in the
    form the kernel evaluates: (A v + B) / (v^2 + E), v = u^2 + D."""
    x = np.expm1((jstar - j) * LNQ) / b
    c1 = a / math.sqrt(math.pi)
    if a >= 1e4:                      # Lorentz limit in u = x / a
        u, A, B, D, E = x / a, c1 / a ** 2, 0.0, 1.0, 0.0
    else:
        u, A, B, D, E = x, c1, c1, a * a - 0.5, 2 * a * a
    v = u * u + D
    return (A * v + B) / (v * v + E)


def cheb(K):
    th = (2 * np.arange(K) + 1) * math.pi / (2 * K)
    return np.cos(th), (-1.0) ** np.arange(K) * np.sin(th)


def quarter_nodes():
    """Positions (points after the tile's first) of the 64 quarter nodes,
    lane l = Chebyshev point l % 16 of quarter l // 16."""
    s, _ = cheb(16)
    half = 0.5 * (QUARTER - 1)
    return np.array([QUARTER * (l // 16) + half + half * s[l % 16] for l in range(64)])


def tile_nodes(K):
    s, _ = cheb(K)
    half = 0.5 * (TILE - 1)
    return half + half * s


def lagrange_at(xq, K):
    """Lagrange basis values of the K whole-tile nodes at points xq
    (barycentric weights, normalised), float64."""
    s, w = cheb(K)
    half = 0.5 * (TILE - 1)
    t = (np.asarray(xq) - half) / half
    r = w[None, :] / (t[:, None] - s[None, :])
    return r / r.sum(axis=1)[:, None]


def quarter_interp_f32(nodes64):
    """The kernel's per-quarter barycentric formula in FP32 at all 1024
    points of the tile from the 64 quarter-node values."""
    s, w = cheb(16)
    s, w = s.astype(F32), w.astype(F32)
    out = np.empty(TILE)
    k = np.arange(QUARTER).astype(F32)
    t = ((k - F32(127.5)) * F32(1.0 / 127.5)).astype(F32)
    for q in range(4):
        f = nodes64[16 * q:16 * q + 16].astype(F32)
        num = np.zeros(QUARTER, F32)
        den = np.zeros(QUARTER, F32)
        for n in range(16):
            r = (w[n] * (F32(1.0) / (t - s[n]))).astype(F32)
            num = (num + r * f[n]).astype(F32)
            den = (den + r).astype(F32)
        out[QUARTER * q:QUARTER * (q + 1)] = (num / den).astype(np.float64)
    return out


def tier_chain_f32(K, jstar, a, b):
    """Tier with K whole-tile nodes: node values (float64 -> FP32), the FP32
    conversion to the quarter nodes, the FP32 quarter interpolation."""
    f = fraction(tile_nodes(K), jstar, a, b).astype(F32)
    V = lagrange_at(quarter_nodes(), K).astype(F32)        # [64 lanes][K]
    acc = np.zeros(64, F32)
    for n in range(K):
        acc = (acc + V[:, n] * f[n]).astype(F32)
    return quarter_interp_f32(acc)


def zone(a, b):
    c1 = LNQ / b
    return math.ceil(15 * 1.02 / c1) + 2 if a < 15 else -1


def worst(K, D, a, b, inside=0.0):
    """Max error relative to the line's part, over the tile, for centres just
    beyond max(D, zone) on either side (fractional parts 0, 1/4, 1/2)."""
    k = np.arange(TILE, dtype=np.float64)
    out = 0.0
    for frac in (0.0, 0.25, 0.5):
        js0 = -float(max(D, zone(a, b)) + 1) - frac + inside
        for js in (js0, TILE - 1 - js0):
            got = tier_chain_f32(K, js, a, b)
            ref = fraction(k, js, a, b)
            out = max(out, float(np.max(np.abs(got - ref) / ref)))
    return out


@pytest.mark.parametrize("K,D", TIERS)
@pytest.mark.parametrize("a", [1e-4, 0.3, 1.0, 5.0, 14.9, 15.0, 100.0, 1e4, 1e5])
@pytest.mark.parametrize("points_per_doppler", [1.0, 1.5, 3.3, 10.0, 30.0, 100.0])
def test_tier_error_bound(K, D, a, points_per_doppler):
    assert worst(K, D, a, points_per_doppler * LNQ) <= BOUND


@pytest.mark.parametrize("K,D", TIERS)
def test_tier_edge_is_probed(K, D):
    """Half the tier's distance breaks its bound for a weakly damped line."""
    assert worst(K, D, 0.3, 1.0 * LNQ, inside=D / 2) > 10 * BOUND


def test_conversion_matrix_is_bounded():
    """No quarter node sits exactly on a whole-tile node (the closest pair,
    for 32 nodes, is 0.002 points apart), and the conversion matrix, computed
    on the host in extended precision, has bounded entries: every row sums
    to 1 and its absolute values to at most the Lebesgue constant (below 3
    for these node counts), so rounding it to FP32 costs at most a few ulp
    of the largest node value."""
    xq = quarter_nodes()
    for K, _ in TIERS:
        gap = np.min(np.abs(xq[:, None] - tile_nodes(K)[None, :]))
        assert gap > 1e-3, (K, gap)
        V = lagrange_at(xq, K)
        assert np.all(np.isfinite(V))
        np.testing.assert_allclose(V.sum(axis=1), 1.0, atol=1e-12)
        assert np.abs(V).sum(axis=1).max() < 3.0

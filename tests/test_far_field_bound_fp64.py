"""The error bound of the plain FP64 path's far field, checked in float64 on
the CPU: a line whose window covers a 1024-point tile, whose |x| < 40 zone
misses it and whose centre lies more than 384 points outside it adds, over
the tile, its four-node Gauss-Hermite pair sum, which the kernel evaluates at
the 16 Chebyshev points of the first kind of each 256-point quarter and
interpolates (barycentric formula).  At the rule's edge the interpolant must
stay within 1e-12 of the four-node sum at every point of the quarter (far
below the FP64 path's per-step tolerance of 1e-9 and the rule's own 3e-12),
for damping from 1e-4 to 1e5 and Doppler widths from 1 to 60 grid points.
The nodes and weights of the rule are numpy's Gauss-Hermite ones, not the
kernel's."""
import math

import numpy as np
import pytest

LNQ = math.log1p(1.0 / 5e5)
NODES = 16
QUARTER = 256
HALF = 0.5 * (QUARTER - 1)
DIST = 384
T4, W4 = np.polynomial.hermite.hermgauss(4)


def gh4(j, jstar, a, b):
    """(a/pi) sum_k w_k / ((x - t_k)^2 + a^2) over the four nodes (S = 1)."""
    x = np.expm1((jstar - j) * LNQ) / np.asarray(b)
    x = np.asarray(x, dtype=np.float64)[..., None]
    return (a / math.pi) * np.sum(W4 / ((x - T4) ** 2 + a * a), axis=-1)


def interpolate(jstar, a, b):
    n = np.arange(NODES)
    th = (2 * n + 1) * math.pi / (2 * NODES)
    s_n, w_n = np.cos(th), (-1.0) ** n * np.sin(th)
    f_n = gh4(HALF + HALF * s_n, jstar, a, b)
    k = np.arange(QUARTER, dtype=np.float64)
    t = (k - HALF) / HALF
    r = w_n[None, :] / (t[:, None] - s_n[None, :])
    return (r @ f_n) / r.sum(axis=1), gh4(k, jstar, a, b)


def closest_allowed_centre(a, b):
    c1 = LNQ / b
    zone = math.ceil(40 * 1.02 / c1) + 2 if a < 40 else -1
    return -float(max(DIST, zone) + 1)


def _worst(a, b):
    worst = 0.0
    for frac in (0.0, 0.25, 0.5):
        jstar = closest_allowed_centre(a, b) - frac
        for js in (jstar, QUARTER - 1 - jstar):
            got, ref = interpolate(js, a, b)
            worst = max(worst, float(np.max(np.abs(got - ref) / ref)))
    return worst


@pytest.mark.parametrize("a", [1e-4, 1e-2, 0.3, 1.0, 5.0, 39.9, 40.0, 100.0, 1e4, 1e5])
@pytest.mark.parametrize("points_per_doppler", [1.0, 1.5, 3.3, 10.0, 30.0, 60.0])
def test_interpolation_error_bound_fp64(a, points_per_doppler):
    assert _worst(a, points_per_doppler * LNQ) <= 1e-12


def test_the_rule_edge_matters():
    """At 192 points instead of 384 the same interpolation errs far more:
    the distance is what the bound rests on."""
    a, b = 0.3, 3.3 * LNQ
    got, ref = interpolate(-193.0, a, b)
    assert np.max(np.abs(got - ref) / ref) > 1e-11

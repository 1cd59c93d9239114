"""The error bound of the mixed path's far field, checked in exact arithmetic
(float64, no GPU): a line whose centre lies as close to a 256-point quarter
as the far-field rule allows (more than 64 points and more than its |x| < 15
zone away) is evaluated at the 16 Chebyshev points of the first kind of the
quarter and interpolated with the barycentric formula.  The interpolant must
stay within 1.5e-5 of the line's two-node fraction at every point of the
quarter (below the fraction's own 5e-5 error at |x| = 15), for damping from
1e-4 to 1e5 (both branches of the fraction) and Doppler widths from 1 to 60
grid points; 40 points further out the error falls below 1e-6.
"""
import math

import numpy as np
import pytest

LNQ = math.log1p(1.0 / 5e5)
NODES = 16
QUARTER = 256
HALF = 0.5 * (QUARTER - 1)
DIST = 64


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


def interpolate(jstar, a, b):
    n = np.arange(NODES)
    th = (2 * n + 1) * math.pi / (2 * NODES)
    s_n, w_n = np.cos(th), (-1.0) ** n * np.sin(th)
    f_n = fraction(HALF + HALF * s_n, jstar, a, b)
    k = np.arange(QUARTER, dtype=np.float64)
    t = (k - HALF) / HALF
    r = w_n[None, :] / (t[:, None] - s_n[None, :])
    return (r @ f_n) / r.sum(axis=1), fraction(k, jstar, a, b)


def closest_allowed_centre(a, b):
    """Centre index just outside the rule, on the low side of [0, 255]."""
    c1 = LNQ / b
    zone = math.ceil(15 * 1.02 / c1) + 2 if a < 15 else -1
    return -float(max(DIST, zone) + 1)


def _worst(a, b, extra=0.0):
    worst = 0.0
    for frac in (0.0, 0.25, 0.5):    # fractional part of the centre
        jstar = closest_allowed_centre(a, b) - frac - extra
        for js in (jstar, QUARTER - 1 - jstar):   # either side of the quarter
            got, ref = interpolate(js, a, b)
            worst = max(worst, float(np.max(np.abs(got - ref) / ref)))
    return worst


@pytest.mark.parametrize("a", [1e-4, 1e-2, 0.3, 1.0, 5.0, 14.9, 15.0, 100.0, 1e4, 1e5])
@pytest.mark.parametrize("points_per_doppler", [1.0, 1.5, 3.3, 10.0, 30.0, 60.0])
def test_interpolation_error_bound(a, points_per_doppler):
    b = points_per_doppler * LNQ
    assert _worst(a, b) <= 1.5e-5
    assert _worst(a, b, extra=40.0) <= 1e-6


def test_interpolation_is_not_trivially_exact():
    """A centre inside the excluded band breaks the bound, so the test above
    does probe the rule's edge."""
    a, b = 0.3, 3.3 * LNQ
    got, ref = interpolate(-10.0, a, b)
    assert np.max(np.abs(got - ref) / ref) > 1e-4

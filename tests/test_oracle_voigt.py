"""Pins of the oracle's Voigt function H(x, a) = Re w(x + ia).

Independent of scipy's Faddeeva routine: closed forms, mpmath's
arbitrary-precision erfc, the Laplace far-wing series, the profile
normalisation and a brute-force quadrature of the defining convolution
integral H = (a/pi) int exp(-t^2) / ((x-t)^2 + a^2) dt.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy.integrate import quad

from oracle import voigt_h

mpmath.mp.dps = 40


def _h_mp(x, a):
    z = mpmath.mpf(x) + 1j * mpmath.mpf(a)
    return float(mpmath.re(mpmath.exp(-z * z) * mpmath.erfc(-1j * z)))


def test_core_value_closed_form():
    # H(0, a) = exp(a^2) erfc(a)
    for a in [1e-9, 1e-5, 1e-2, 0.3, 1.0, 3.7, 12.0, 150.0, 1e4, 1e8, 1e11]:
        ref = float(mpmath.exp(mpmath.mpf(a) ** 2) * mpmath.erfc(mpmath.mpf(a)))
        assert voigt_h(0.0, a) == pytest.approx(ref, rel=1e-13)


def test_gaussian_limit():
    x = np.linspace(0.0, 26.0, 400)
    np.testing.assert_allclose(voigt_h(x, 0.0), np.exp(-x * x), rtol=1e-13, atol=0)


def test_far_wing_series():
    # Laplace asymptotic series of Re w for |z| -> infinity, small a:
    # H ~ a/(sqrt(pi) x^2) (1 + 3/(2x^2) + 15/(4x^4) + ...)
    for x in [60.0, 120.0, 500.0]:
        for a in [1e-9, 1e-4, 1e-2]:
            s = 1.0 + 1.5 / x ** 2 + 15.0 / (4 * x ** 4)
            ref = a / (math.sqrt(math.pi) * x * x) * s
            assert voigt_h(x, a) == pytest.approx(ref, rel=1e-9)


@pytest.mark.parametrize("a", [1e-3, 0.1, 1.0, 5.0])
def test_profile_normalisation(a):
    # int H dx over the real line = sqrt(pi) (area of the profile)
    f = lambda x: float(voigt_h(x, a))
    tail = 2.0 * a / (math.sqrt(math.pi) * 2000.0)  # Lorentz tail beyond |x| = 2000
    val = 2.0 * sum(quad(f, lo, hi, limit=400, epsabs=1e-14, epsrel=1e-13)[0]
                    for lo, hi in [(0, 1), (1, 5), (5, 50), (50, 2000)])
    assert val + tail == pytest.approx(math.sqrt(math.pi), rel=2e-8)


def test_brute_force_convolution():
    rng = np.random.default_rng(11)
    for _ in range(12):
        x = float(rng.uniform(0.0, 8.0))
        a = float(10 ** rng.uniform(-1.5, 1.0))
        f = lambda t: mpmath.exp(-t * t) / ((x - t) ** 2 + a * a)
        ref = float(a / mpmath.pi * mpmath.quad(f, [-mpmath.inf, x - 1, x, x + 1, mpmath.inf]))
        assert voigt_h(x, a) == pytest.approx(ref, rel=1e-10)


def test_mpmath_random_points():
    rng = np.random.default_rng(5)
    xs = np.concatenate([rng.uniform(0, 20, 80), 10 ** rng.uniform(-3, 2.7, 80)])
    As = 10 ** rng.uniform(-9, 11, xs.size)
    for x, a in zip(xs, As):
        assert voigt_h(x, a) == pytest.approx(_h_mp(x, a), rel=1e-12)


def test_symmetric_and_positive():
    xp = np.linspace(0, 40, 401)
    for a in [1e-6, 0.05, 2.0]:
        hp, hm = voigt_h(xp, a), voigt_h(-xp, a)
        assert np.all(hp > 0)
        np.testing.assert_allclose(hp, hm, rtol=1e-14)

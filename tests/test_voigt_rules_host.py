"""Error bounds of the Voigt kernels' evaluation rules, checked on the host.

Each rule is written here as the kernels evaluate it, with its nodes and
weights built independently (numpy's Gauss-Hermite nodes, trapezoid weights
(h/pi) e^{-t^2} from their definition), in float64, and compared with the
Voigt function H(x, a) = Re w(x + i a) (scipy's Faddeeva function for the
FP32 rules; mpmath at 30 digits for the FP64 rules and the series, whose
bounds lie below scipy's own accuracy) over the region where the kernels use
the rule.  The bounds are the ones the kernels' designs rest on:

  FP32  two-node pair fraction      |z| >= 15                5e-5
        the same, Lorentz limit     a >= 1e4                 1/(2 a^2)
        four-node pair sum          |z| >= 6                 2e-5
        pole-corrected trapezoid    a in [0.4, 15), |x| <= 70   5e-6
        (h = 0.75, 13 nodes, |t| <= 4.2)
        small-damping series        a < 0.4, any x           1e-5
  FP64  four-node pair sum          |z| >= 40                3e-12
        eight-node pair sum         8 <= |z| < 40            2e-11 (5e-13 from |z| = 10)
        pole-corrected trapezoid    |z| < 8                  2e-13
        (h = 0.55, 23 nodes, |t| <= 5.9)

(The rounding of the FP32 kernels adds a few ulp on top; the GPU tests
compare their output with the oracle end to end.)
"""
import math

import mpmath
import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from scipy.special import wofz

SQRT_PI = math.sqrt(math.pi)


def H(x, a):
    return wofz(np.asarray(x) + 1j * np.asarray(a)).real


def H_mp(x, a):
    z = mpmath.mpc(x, a)
    return float(mpmath.re(mpmath.exp(-z * z) * mpmath.erfc(-1j * z)))


def pair_sum(x, a, n):
    """n-node Gauss-Hermite rule for H = (a/pi) int e^{-t^2} / ((x-t)^2 + a^2) dt,
    the +-t_k terms of each node pair combined into one fraction
    2 p / (p^2 - 4 t^2 x^2), p = x^2 + a^2 + t^2."""
    t, w = hermgauss(n)
    t, w = t[t > 0], w[t > 0]
    x = np.asarray(x, dtype=np.float64)[..., None]
    a = np.asarray(a, dtype=np.float64)[..., None]
    p = x * x + a * a + t * t
    d = p * p - 4.0 * t * t * x * x
    return (2.0 * a[..., 0] / math.pi) * np.sum(w * p / d, axis=-1)


def two_node_fraction(x, a):
    """(A v + B) / (v^2 + E), v = x^2 + D, with A = B = a / sqrt(pi),
    D = a^2 - 1/2, E = 2 a^2 (the far-wing record of the mixed path, S = 1)."""
    A = a / SQRT_PI
    v = x * x + a * a - 0.5
    return (A * v + A) / (v * v + 2.0 * a * a)


def trapezoid(x, a, h, half, tmax):
    """Pole-corrected trapezoidal rule on nodes t = (k + delta) h, k = -half..half,
    delta = 1/2 where x / h lies within 1/4 of an integer; weights (h/pi) e^{-t^2}
    for |t| <= tmax; the residue term Re[2 e^{-z^2} / (1 -+ e^{-2 pi i z/h})]
    added for a < pi / h (as the kernels evaluate it)."""
    hx = x / h
    fr = hx - np.rint(hx)
    sh = np.abs(fr) < 0.25
    delta = np.where(sh, 0.5, 0.0)
    v = np.zeros_like(x)
    for k in range(-half, half + 1):
        t = (k + delta) * h
        c = np.where(np.abs(t) <= tmax, h / math.pi * np.exp(-t * t), 0.0)
        v += a * c / ((x - t) ** 2 + a * a)
    e2 = 2.0 * math.pi * a / h
    mag = np.exp(a * a - x * x - e2)
    ep = np.exp(-e2)
    ph, th = 2.0 * math.pi * hx, 2.0 * math.pi * hx - 2.0 * x * a
    sgn = np.where(sh, 1.0, -1.0)
    dre, dim = ep * np.cos(ph) + sgn, ep * np.sin(ph)
    corr = 2.0 * mag * (np.cos(th) * dre + np.sin(th) * dim) / (dre * dre + dim * dim)
    return v + np.where(a < math.pi / h, corr, 0.0)


def rel(got, ref):
    return np.max(np.abs(np.asarray(got) / np.asarray(ref) - 1.0))


def _polar(rmin, rmax, amin, amax, n_r=60, n_t=60):
    """(x, a) with |x + i a| from rmin to rmax (log-spaced), a in [amin, amax]."""
    r = np.geomspace(rmin, rmax, n_r)[:, None]
    th = np.linspace(0.0, math.pi / 2, n_t)[None, :]
    x, a = (r * np.cos(th)).ravel(), (r * np.sin(th)).ravel()
    keep = (a >= amin) & (a < amax)
    return x[keep], a[keep]


def test_fp32_two_node_fraction():
    x, a = _polar(15.0, 1e4, 1e-4, 1e4)
    assert x.size > 1000
    assert rel(two_node_fraction(x, a), H(x, a)) <= 5e-5
    # the rule does not hold inside |z| = 15 (so the zone is needed)
    x, a = _polar(6.0, 10.0, 1e-4, 10.0)
    assert rel(two_node_fraction(x, a), H(x, a)) > 2e-4


def test_fp32_lorentz_limit():
    for a in (1e4, 3e4, 1e5, 1e6):
        x = a * np.concatenate([[0.0], np.geomspace(1e-3, 1e3, 200)])
        u = x / a
        got = (a / SQRT_PI / (a * a)) / (u * u + 1.0)
        assert rel(got, H(x, a)) <= 1.0 / (2.0 * a * a) + 1e-12


def test_fp32_four_node_pair_sum():
    x, a = _polar(6.0, 300.0, 1e-4, 300.0)
    assert rel(pair_sum(x, a, 4), H(x, a)) <= 2e-5
    # and it is the rule of the two-node fraction with two more nodes
    assert rel(pair_sum(x, a, 2), two_node_fraction(x, a)) <= 1e-12


@pytest.mark.parametrize("a", [0.4, 0.6, 1.0, 2.0, 3.5, 4.18, 4.2, 6.0, 10.0, 14.9])
def test_fp32_trapezoid(a):
    # core rows reach |x| = 6 + 64 points, up to about 70 Doppler widths at one point per width
    x = np.concatenate([np.linspace(0.0, 70.0, 7001), np.linspace(0.0, 3.0, 401) + 1e-3])
    got = trapezoid(x, np.full_like(x, a), 0.75, 6, 4.2)
    assert rel(got, H(x, np.full_like(x, a))) <= 5e-6


def _series_terms(a):
    return 1 if a < 0.004 else (2 if a < 0.06 else (3 if a < 0.2 else 4))


def _T(n, x):
    """T_n(x) = Re(i^n w^(n)(x)) / n!, the coefficient of a^n in Re w(x + i a)."""
    w = lambda t: mpmath.exp(-t * t) * mpmath.erfc(-1j * t)
    return float(mpmath.re((1j) ** n * mpmath.diff(w, x, n)) / mpmath.factorial(n))


@pytest.mark.parametrize("a", [1e-5, 3e-3, 0.0039, 0.05, 0.059, 0.15, 0.199, 0.3, 0.399])
def test_fp32_small_damping_series(a):
    """H = e^{a^2 - x^2} cos 2xa + sum_{k < nt} a^{2k+1} T_{2k+1}(x), nt from a."""
    mpmath.mp.dps = 30
    nt = _series_terms(a)
    worst = 0.0
    for x in [0.0, 0.3, 0.7, 1.0, 1.5, 2.0, 2.5, 3.0, 4.0, 5.0, 7.0, 10.0, 15.0, 30.0, 100.0]:
        s = math.exp(a * a - x * x) * math.cos(2.0 * x * a)
        s += sum(a ** (2 * k + 1) * _T(2 * k + 1, mpmath.mpf(x)) for k in range(nt))
        worst = max(worst, abs(s / H_mp(x, a) - 1.0))
    assert worst <= 1e-5, worst


def _mp_rel(fn, pts):
    mpmath.mp.dps = 30
    return max(abs(fn(x, a) / H_mp(x, a) - 1.0) for x, a in pts)


def test_fp64_four_node_pair_sum():
    x, a = _polar(40.0, 1e4, 1e-4, 1e4, n_r=12, n_t=12)
    assert _mp_rel(lambda x, a: float(pair_sum(x, a, 4)), zip(x, a)) <= 3e-12


def test_fp64_eight_node_pair_sum():
    x, a = _polar(8.0, 40.0, 1e-4, 40.0, n_r=12, n_t=12)
    assert _mp_rel(lambda x, a: float(pair_sum(x, a, 8)), zip(x, a)) <= 2e-11
    x, a = _polar(10.0, 40.0, 1e-4, 40.0, n_r=10, n_t=10)
    assert _mp_rel(lambda x, a: float(pair_sum(x, a, 8)), zip(x, a)) <= 5e-13


def test_fp64_trapezoid():
    pts = [(x, a) for x in np.linspace(0.0, 8.0, 17) for a in (1e-4, 0.01, 0.3, 1.0, 3.0, 5.6, 5.8, 7.9)
           if math.hypot(x, a) < 8.0]
    fn = lambda x, a: float(trapezoid(np.array([x]), np.array([a]), 0.55, 11, 5.9)[0])
    assert _mp_rel(fn, pts) <= 2e-13

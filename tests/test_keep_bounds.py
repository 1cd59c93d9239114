"""The selection kernel decides most keep tests S erfcx(a) >= thr from the
bounds 2/(sqrt(pi)(a + sqrt(a^2 + 2))) < erfcx(a) <= 2/(sqrt(pi)(a +
sqrt(a^2 + 4/pi))) (Abramowitz and Stegun 7.1.13) and calls erfcx only in
between.  Checked here against scipy's erfcx over the damping range of the
workloads and beyond, with the kernel's decision rule replayed in float64:
its decisions equal the exact test's except within 1e-12 of the threshold."""
import math

import numpy as np
from scipy.special import erfcx

SQRT_PI = math.sqrt(math.pi)


def bounds(a):
    lo = 2.0 / (SQRT_PI * (a + np.sqrt(a * a + 2.0)))
    hi = 2.0 / (SQRT_PI * (a + np.sqrt(a * a + 4.0 / math.pi)))
    return lo, hi


def keep(S, a, thr):
    lo, hi = bounds(a)
    out = np.where(S * lo >= thr * (1 + 1e-13), True,
                   np.where(S * hi < thr * (1 - 1e-13), False, S * erfcx(a) >= thr))
    return np.where(S >= thr, out, False)


def test_bounds_hold():
    a = np.concatenate([[0.0], np.logspace(-12, 11, 200001)])
    e = erfcx(a)
    lo, hi = bounds(a)
    assert np.all(lo < e * (1 + 1e-15))
    assert np.all(hi >= e * (1 - 1e-15))
    # the undecided band: at most sqrt(pi/2) = 1.2533 wide in S (at a = 0),
    # narrowing as 1 + (1 - 2/pi) / (2 a^2) for large a
    gap = hi / lo
    assert gap.max() <= math.sqrt(math.pi / 2.0) * (1 + 1e-14)
    mid = (a > 10) & (a < 1e5)
    assert np.all((gap[mid] - 1) * a[mid] ** 2 < (1 - 2 / math.pi) / 2 * 1.01)


def test_decisions_match_the_exact_test():
    rng = np.random.default_rng(0)
    n = 2_000_000
    a = 10.0 ** rng.uniform(-9, 9, n)
    thr = 10.0 ** rng.uniform(-8, 2, n)
    # strengths spread around the threshold, many inside the bounds' gap
    S = thr / erfcx(a) * 10.0 ** rng.uniform(-0.3, 0.3, n)
    exact = S * erfcx(a) >= thr
    got = keep(S, a, thr)
    diff = got != exact
    near = np.abs(S * erfcx(a) / thr - 1.0) < 1e-12
    assert not np.any(diff & ~near)
    assert np.mean(S * bounds(a)[0] >= thr * (1 + 1e-13)) > 0.3     # the bounds decide most

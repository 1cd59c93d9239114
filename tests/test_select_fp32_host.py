"""The selection's FP32 keep test, checked on the host (no GPU).

The selection kernel decides the keep test S erfcx(a) >= thr in FP32 first:
the classical erfcx bounds evaluated in FP32 settle every line whose
S erfcx(a) / thr is more than 1e-5 away from 1, and the FP64 test takes the
rest.  This test runs the same FP32 operations in numpy float32 (one
rounding per operation; the square roots, which the kernel takes from the
hardware within 1 ulp, moved by a random ulp) on lines spread around the
keep boundary (damping 1e-5 to 1e5, half of them within 1e-3 of it):
wherever the FP32 test
decides, its decision must equal the exact one (scipy's erfcx, Sec. 2.1 and
App. E); and it must decide for most lines, or it would not pay.
"""
import math

import numpy as np
from scipy.special import erfcx

F = np.float32


def fmaf(a, b, c):
    return F(np.float64(a) * np.float64(b) + np.float64(c))


def sqrt1ulp(x, rng=np.random.default_rng(7)):
    """FP32 square root within 1 ulp (the hardware's v_sqrt_f32): the
    correctly rounded root moved by a random -1, 0 or +1 ulp."""
    s = np.sqrt(F(x))
    return np.nextafter(s, F(np.inf) if rng.random() < 0.5 else F(0)) if rng.random() < 2 / 3 else s


def keep32(rf, af):
    """keep_line32: 1 keep, 0 drop, -1 undecided."""
    rf, af = F(rf), F(af)
    if not (rf < F(1e30) and af < F(1e15)):
        return -1
    sp = F(1.77245385)
    r2 = F(2.0) * rf
    if r2 >= (F(1.0) + F(1e-5)) * sp * (af + sqrt1ulp(fmaf(af, af, 2.0))):
        return 1
    if r2 < (F(1.0) - F(1e-5)) * sp * (af + sqrt1ulp(fmaf(af, af, F(4.0 / math.pi)))):
        return 0
    return -1


def test_keep_decisions_equal_fp64():
    rng = np.random.default_rng(12)
    n = 200_000
    a = 10.0 ** rng.uniform(-5, 5, n)
    # ratios r erfcx(a) spread around 1, many within 1e-3 of it
    q = np.where(rng.random(n) < 0.5, 10.0 ** rng.uniform(-3, 3, n), 1.0 + rng.uniform(-1e-3, 1e-3, n))
    thr = 10.0 ** rng.uniform(-8, 2, n)
    S = q / erfcx(a) * thr
    decided = 0
    for k in range(n):
        d = keep32(F(S[k] * (1.0 / thr[k])), a[k])
        if d < 0:
            continue
        decided += 1
        exact = S[k] * erfcx(a[k]) >= thr[k]
        assert bool(d) == bool(exact), (S[k], a[k], thr[k])
    assert decided > 0.45 * n


def test_keep_leaves_out_of_range_inputs_to_fp64():
    """Damping or strength ratios beyond the FP32 ranges the bounds assume
    (a^2 would overflow) are left to the FP64 test, never decided here."""
    for rf, af in ((1e25, 1e19), (1e31, 1.0), (np.inf, 1.0), (2.0, 3e38)):
        assert keep32(F(rf), af) == -1


def log1p_pm(v):
    """ln(1 + v) and ln(1 - v) from the odd and even parts of the series of
    ln(1 + v), as the selection evaluates them for |v| <= 1/16 (odd part to
    v^13, even part to v^12, Horner in v^2)."""
    w = v * v
    o = 1.0 / 13
    for c in (11, 9, 7, 5, 3, 1):
        o = o * w + 1.0 / c
    o = o * v
    e = 1.0 / 12
    for c in (10, 8, 6, 4, 2):
        e = e * w + 1.0 / c
    e = -e * w
    return e + o, e - o


def test_log1p_pair_series():
    """Within 4 ulp of the library log1p over |v| <= 1/16 (edges of the
    window move by at most that times their distance from the centre, far
    below the 1e-7 points where a window edge counts as a tie)."""
    v = np.concatenate([np.linspace(-1.0 / 16, 1.0 / 16, 200001), np.geomspace(1e-12, 1.0 / 16, 2001)])
    v = v[v != 0.0]
    lp, lm = log1p_pm(v)
    assert np.max(np.abs(lp / np.log1p(v) - 1.0)) <= 4 * 2.0 ** -52
    assert np.max(np.abs(lm / np.log1p(-v) - 1.0)) <= 4 * 2.0 ** -52
    assert log1p_pm(0.0) == (0.0, 0.0)

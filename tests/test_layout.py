"""Grid size and bin layouts (App. E grid formula; user-defined binning)."""
import json
import math
import os

import mpmath
import numpy as np

import oracle
from paper_2105_13611_amd import workload as W

FACTS = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_facts.json")))


def _n_mp(lf, ll, R):
    mpmath.mp.dps = 50
    q = 1 + mpmath.mpf(1) / R
    n = int(mpmath.floor(mpmath.log(mpmath.mpf(ll) / mpmath.mpf(lf)) / mpmath.log(q))) + 1
    # brute-force edge check in 50-digit arithmetic: lambda_{N-1} <= ll < lambda_N
    assert mpmath.mpf(lf) * q ** (n - 1) <= mpmath.mpf(ll) < mpmath.mpf(lf) * q ** n
    return n


def test_grid_sizes():
    R = FACTS["resolving_power"]["value"]
    lf = FACTS["grid_lambda_first_nm"]["value"]
    ll = FACTS["grid_lambda_last_nm"]["value"]
    assert _n_mp(300.0, 310.0, R) == 16395
    assert _n_mp(lf, ll, R) == 3507864
    for a, b in [(300.0, 310.0), (lf, ll), (498.0, 502.0), (9.0, 9.1)]:
        n = _n_mp(a, b, R)
        assert oracle.grid_size(a, b, R) == n
        assert W.grid_size(a, b, R) == n


def test_brute_force_small_grid():
    # count lambda_first q^j <= lambda_last by stepping in exact rationals
    from fractions import Fraction
    lf, ll, R = Fraction(300), Fraction(30003, 100), 500000
    q = 1 + Fraction(1, R)
    n, lam = 0, lf
    while lam <= ll:
        n += 1
        lam *= q
    assert oracle.grid_size(300.0, 300.03, float(R)) == n


def test_cfg1_bins():
    w = W.config(1)
    e = w.layout.bin_edges
    d = np.diff(e)
    assert e[0] == 0 and e[-1] == 16395 and len(d) == 20
    assert set(d.tolist()) == {819, 820}
    assert len(w.layout.step_frac) == FACTS["n_standard_subbins"]["value"]
    assert math.isclose(w.layout.step_frac.sum(), 1.0, rel_tol=1e-12)


def test_ramp_bins():
    N = 3507864
    e = W.ramp_bins(N, 1212)
    d = np.diff(e)
    assert e[0] == 0 and e[-1] == N and len(d) == 1212
    assert d.min() == 500 and d.max() == 8795
    assert np.all(np.diff(d) >= 0)


def test_tp_grid_shape():
    p = W.dfsynthe_tp_grid()
    assert p.n_points == FACTS["n_temperatures"]["value"] * FACTS["n_pressures"]["value"]
    assert p.log10_P.min() == FACTS["log10_p_min"]["value"] and p.log10_P.max() == FACTS["log10_p_max"]["value"]
    assert math.isclose(p.T_K.min(), 2000.0) and math.isclose(p.T_K.max(), 200000.0)

"""Pins of the ODF reduction (Sec. 2.3: sort ascending, sub-bins given as
fractions of the bin, geometric or arithmetic sub-bin means)."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle.odf import odf_reduce_bin

STEPS12 = np.array([0.1] * 9 + [0.05, 0.04, 0.01])


def _brute(values, fracs, mean):
    """Exact rational weights: sorted point i covers [i, i+1); sub-bin s
    covers [F_{s-1} n, F_s n) with F from exact fractions."""
    v = sorted(values)
    n = len(v)
    fr = [Fraction(f).limit_denominator(10 ** 6) for f in fracs]
    tot = sum(fr)
    F = [Fraction(0)]
    for f in fr:
        F.append(F[-1] + f / tot)
    out = []
    for s in range(len(fr)):
        lo, hi = F[s] * n, F[s + 1] * n
        acc = 0.0
        for i, x in enumerate(v):
            w = max(Fraction(0), min(Fraction(i + 1), hi) - max(Fraction(i), lo))
            if w:
                acc += float(w) * (math.log(x) if mean == "geometric" else x)
        m = acc / float(hi - lo)
        out.append(math.exp(m) if mean == "geometric" else m)
    return np.array(out)


@pytest.mark.parametrize("mean", ["geometric", "arithmetic"])
def test_brute_force_tiny_bins(mean):
    rng = np.random.default_rng(3)
    for nb in range(1, 21):
        for fr in (STEPS12, np.array([0.5, 0.3, 0.2]), np.array([1.0])):
            v = 10 ** rng.uniform(-5, 5, nb)
            np.testing.assert_allclose(odf_reduce_bin(v, fr, mean), _brute(v, fr, mean), rtol=1e-12)


@pytest.mark.parametrize("mean", ["geometric", "arithmetic"])
def test_invariants(mean):
    rng = np.random.default_rng(4)
    for nb in [1, 7, 37, 819, 820, 8795]:
        v = 10 ** rng.uniform(-6, 6, nb)
        s = odf_reduce_bin(v, STEPS12, mean)
        assert np.all(np.diff(s) >= -1e-12 * np.abs(s[1:]))          # monotone steps
        if mean == "geometric":
            assert np.sum(STEPS12 * np.log(s)) == pytest.approx(np.mean(np.log(v)), rel=1e-12, abs=1e-12)
        else:
            assert np.sum(STEPS12 * s) == pytest.approx(np.mean(v), rel=1e-12)
        perm = rng.permutation(nb)
        np.testing.assert_allclose(odf_reduce_bin(v[perm], STEPS12, mean), s, rtol=1e-14)
        np.testing.assert_allclose(odf_reduce_bin(np.full(nb, 3.25), STEPS12, mean), 3.25, rtol=1e-14)
        one = odf_reduce_bin(v, np.array([1.0]), mean)[0]
        ref = math.exp(np.mean(np.log(v))) if mean == "geometric" else np.mean(v)
        assert one == pytest.approx(ref, rel=1e-12)
        # extreme steps bracket the data
        assert s[0] >= v.min() * (1 - 1e-12) and s[-1] <= v.max() * (1 + 1e-12)


def test_point_odf_cfg1_properties(cfg1):
    w = cfg1
    steps, cnt, ex = oracle.odf_point(w.lines, w.species, w.species.abundance, 5000.0, 4.0, 2.0,
                                      w.layout, w.options, bins=[0, 7, 19], return_fine=True)
    assert steps.shape == (3, 12)
    assert np.all(np.diff(steps, axis=1) >= 0)
    for k, b in enumerate([0, 7, 19]):
        kl, kt = ex["fine"][b]
        assert np.sum(w.layout.step_frac * np.log(steps[k])) == pytest.approx(np.mean(np.log(kt)), rel=1e-12)
    assert cnt["line_evals"] == 10000 and 0 < cnt["survivors"] <= 10000


def test_duplicated_lines_double_opacity(cfg1):
    from paper_2105_13611_amd import workload as W
    w = cfg1
    idx = np.arange(500)
    l1 = w.lines.take(idx)
    l2 = w.lines.take(np.concatenate([idx, idx]))
    b = [3]
    o = W.Options(cutoff=1e-4)
    _, _, e1 = oracle.odf_point(l1, w.species, w.species.abundance, 5000.0, 4.0, 2.0, w.layout, o, b, True)
    _, _, e2 = oracle.odf_point(l2, w.species, w.species.abundance, 5000.0, 4.0, 2.0, w.layout, o, b, True)
    k1 = e1["fine"][3][0]
    k2 = e2["fine"][3][0]
    # doubling every line doubles kappa_l where the windows are unchanged
    # (a line at twice the strength may widen its window; compare where both are nonzero)
    m = k1 > 0
    ratio = k2[m] / k1[m]
    assert np.median(ratio) == pytest.approx(2.0, rel=1e-12)


@pytest.mark.parametrize("mean", ["geometric", "arithmetic"])
def test_fine_table_is_the_odf_of_one_point_bins(cfg1, mean):
    # Sec. 4.1: the pre-tabulated opacity is an ODF whose bins are single
    # fine points with one sub-bin
    from dataclasses import replace
    from paper_2105_13611_amd import workload as W
    w = cfg1
    N = oracle.grid_size(w.layout.lambda_first_nm, w.layout.lambda_last_nm, w.layout.resolving_power)
    one = W.Layout(w.layout.lambda_first_nm, w.layout.lambda_last_nm, w.layout.resolving_power,
                   np.arange(N + 1, dtype=np.int64), np.array([1.0]))
    opts = replace(w.options, mean=mean)
    fine, lq = oracle.fine_table_point(w.lines, w.species, w.species.abundance, 5000.0, 4.0, 2.0,
                                       w.layout, opts)
    assert fine.shape == (N,)
    assert np.all(fine >= opts.cutoff * oracle.physics.kappa_c(oracle.grid_lambda_nm(w.layout, np.arange(N)), opts))
    bins = np.unique(np.linspace(0, N - 1, 150).astype(np.int64))
    steps, _, _ = oracle.odf_point(w.lines, w.species, w.species.abundance, 5000.0, 4.0, 2.0,
                                   one, opts, bins=bins)
    # (the ODF sums each bin's lines on their own: same terms, another order)
    np.testing.assert_allclose(steps[:, 0], fine[bins], rtol=1e-13)
    # a window of the grid is the same slice of the whole (up to the order
    # in which the lines are summed)
    part, _ = oracle.fine_table_point(w.lines, w.species, w.species.abundance, 5000.0, 4.0, 2.0,
                                      w.layout, opts, 4000, 4100)
    np.testing.assert_allclose(part, fine[4000:4100], rtol=1e-13)


COLUMNS = np.array([1e-3, 1e-2, 0.1, 1.0, 10.0, 100.0])


def test_slab_constant_bin_is_exact():
    # a flat bin: every sub-bin mean is the value, so any ODF is exact
    v = np.full(500, 37.5)
    for fr in (STEPS12, np.array([0.9, 0.1]), np.array([0.5, 0.3, 0.15, 0.05])):
        for mean in ("geometric", "arithmetic"):
            st = odf_reduce_bin(v, fr, mean)
            np.testing.assert_allclose(oracle.slab_odf_intensity(st, fr, 0.4, COLUMNS),
                                       oracle.slab_fine_intensity(v, 0.4, COLUMNS), rtol=1e-14)


def test_slab_one_point_sub_bins_reproduce_the_fine_grid():
    rng = np.random.default_rng(11)
    v = 10.0 ** rng.uniform(-3, 5, 40)
    fr = np.full(40, 1.0 / 40)
    for mean in ("geometric", "arithmetic"):
        st = odf_reduce_bin(v, fr, mean)
        np.testing.assert_allclose(oracle.slab_odf_intensity(st, fr, 0.3, COLUMNS),
                                   oracle.slab_fine_intensity(v, 0.3, COLUMNS), rtol=1e-12)


def test_slab_thin_and_thick_limits():
    rng = np.random.default_rng(12)
    v = 10.0 ** rng.uniform(-2, 4, 1000)
    fr = np.array([0.7, 0.2, 0.08, 0.02])
    thin = np.array([1e-12])
    ar = odf_reduce_bin(v, fr, "arithmetic")
    ge = odf_reduce_bin(v, fr, "geometric")
    ref = oracle.slab_fine_intensity(v, 0.5, thin)
    # optically thin: I is linear in kappa, so the arithmetic mean is exact
    # and the geometric mean (below the arithmetic one) under-estimates
    assert oracle.slab_odf_intensity(ar, fr, 0.5, thin)[0] == pytest.approx(ref[0], rel=1e-9)
    assert oracle.slab_odf_intensity(ge, fr, 0.5, thin)[0] < ref[0] * (1 - 1e-3)
    # optically thick: every form saturates at the Planck function
    thick = np.array([1e6])
    assert oracle.slab_odf_intensity(ge, fr, 0.5, thick)[0] == pytest.approx(1.0, abs=1e-12)
    assert oracle.slab_fine_intensity(v, 0.5, thick)[0] == pytest.approx(1.0, abs=1e-12)

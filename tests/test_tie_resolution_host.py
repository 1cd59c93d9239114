"""Host logic of the GPU tests' tie handling (no GPU): a bin's reference
recomputed with another side's keep and window decisions.

Decisions equal to the oracle's give the oracle's steps exactly; a window
edge that sits within rounding of an integer may move by one point and the
reference follows it; any other difference is rejected."""
import numpy as np
import pytest

import oracle
from paper_2105_13611_amd import workload as W
from tests.gpu_helpers import oracle_bin_with_gpu_decisions


def _decisions(lq, surv=None, jlo=None, jhi=None):
    surv = lq["surv"] if surv is None else surv
    idx = np.nonzero(surv)[0]
    return dict(orig=idx.astype(np.int64),
                jlo=(lq["jlo"] if jlo is None else jlo)[idx].astype(np.int64),
                jhi=(lq["jhi"] if jhi is None else jhi)[idx].astype(np.int64))


@pytest.fixture(scope="module")
def case():
    w = W.config(1, n_lines=2000)
    steps, _, ex = oracle.odf_point(w.lines, w.species, w.species.abundance, 5000.0, 4.0, 2.0,
                                    w.layout, w.options)
    return w, steps, ex["lq"]


def test_own_decisions_reproduce_the_oracle(case):
    w, steps, lq = case
    dec = _decisions(lq)
    for b in (0, 7, 19):
        got = oracle_bin_with_gpu_decisions(lq, w.layout, w.options, b, dec)
        np.testing.assert_array_equal(got, steps[b])


def test_a_tie_edge_may_move_by_one(case):
    w, steps, lq = case
    e = w.layout.bin_edges
    b = 7
    # a kept line whose window starts inside bin 7: make its real start a tie
    i = int(np.nonzero(lq["surv"] & (lq["jlo"] > e[b] + 2) & (lq["jlo"] < e[b + 1] - 2))[0][0])
    lq2 = dict(lq)
    lq2["jlo_r"] = lq["jlo_r"].copy()
    lq2["jlo_r"][i] = float(lq["jlo"][i]) - 1e-9      # ceil gives jlo; within rounding, jlo + 1
    jlo = lq["jlo"].copy()
    jlo[i] += 1                                         # the other side took the other integer
    got = oracle_bin_with_gpu_decisions(lq2, w.layout, w.options, b, _decisions(lq, jlo=jlo))
    lq3 = dict(lq)
    lq3["jlo"] = jlo
    j0, j1 = int(e[b]), int(e[b + 1])
    kt = np.maximum(oracle.fine_opacity(lq3, w.layout, j0, j1),
                    w.options.cutoff * oracle.physics.kappa_c(oracle.grid_lambda_nm(w.layout, np.arange(j0, j1)), w.options))
    ref = oracle.odf_reduce_bin(kt, w.layout.step_frac, w.options.mean)
    np.testing.assert_array_equal(got, ref)
    assert not np.array_equal(got, steps[b])
    # the tie allows jlo and jlo + 1 only
    jlo[i] = lq["jlo"][i] - 1
    with pytest.raises(AssertionError, match="window starts"):
        oracle_bin_with_gpu_decisions(lq2, w.layout, w.options, b, _decisions(lq, jlo=jlo))


def test_differences_away_from_a_tie_are_rejected(case):
    w, steps, lq = case
    e = w.layout.bin_edges
    b = 7
    i = int(np.nonzero(lq["surv"] & (lq["jlo"] > e[b] + 2) & (lq["jlo"] < e[b + 1] - 2))[0][0])
    jlo = lq["jlo"].copy()
    jlo[i] += 1
    with pytest.raises(AssertionError, match="window starts"):
        oracle_bin_with_gpu_decisions(lq, w.layout, w.options, b, _decisions(lq, jlo=jlo))
    surv = lq["surv"].copy()
    surv[i] = False
    with pytest.raises(AssertionError, match="keep decisions"):
        oracle_bin_with_gpu_decisions(lq, w.layout, w.options, b, _decisions(lq, surv=surv))

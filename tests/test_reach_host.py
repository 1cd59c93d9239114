"""The per-point line reach used to cut the oracle's work at large sizes
(tests/gpu_helpers.Reach) keeps every line whose window touches a bin."""
import numpy as np
import pytest

import oracle
from paper_2105_13611_amd import workload as W
from tests.gpu_helpers import Reach


@pytest.fixture(scope="module")
def sample():
    w = W.config(2)
    rng = np.random.default_rng(7)
    take = np.sort(rng.choice(w.lines.n_lines, 200_000, replace=False))
    return w, w.lines.take(take)


@pytest.mark.parametrize("T,logP,v", [(2000.0, -4.0, 0.0), (5000.0, 4.0, 2.0), (20000.0, 8.0, 2.0),
                                      (200000.0, 0.0, 8.0)])
def test_reach_is_a_superset(sample, T, logP, v):
    w, lines = sample
    bins = [int(b) for b in np.round(np.linspace(0, w.layout.n_bins - 1, 64))]
    lq = oracle.line_quantities(lines, w.species, w.species.abundance, T, logP, v, w.layout, w.options)
    e = w.layout.bin_edges
    need = np.zeros(lines.n_lines, dtype=bool)
    s = lq["surv"]
    for b in bins:
        need |= s & (lq["jlo"] < e[b + 1]) & (lq["jhi"] >= e[b])
    got = np.zeros(lines.n_lines, dtype=bool)
    got[Reach(lines, w.species, w.layout, w.options).lines_for(bins, T, v)] = True
    assert need.sum() > 0
    assert np.all(got[need]), f"{int((need & ~got).sum())} lines reach a bin outside the subset"
    # and it is a real cut at cool points
    if T <= 5000.0:
        assert got.sum() < 0.5 * lines.n_lines

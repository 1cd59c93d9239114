"""Parity at the benchmark's full size, on sampled outputs.

The full 1e7-line list, the 3 507 864-point grid and the 1212-bin ramp of the
benchmark table, computed with the benchmark's workspace (64-point device
batches), at sampled (T, P, v_turb) points that span the grid's cost range;
the oracle checks a few bins of each (it needs minutes per point for all).
"""
import numpy as np
import pytest

import oracle
from paper_2105_13611_amd import workload as W
from tests.gpu_helpers import ambiguous_bins, log10_err, rel_err

pytestmark = pytest.mark.gpu

# the benchmark's workspace; the batch then holds all sampled points
WORKSPACE = 40 << 30
POINTS = W.Points(np.array([5000.0, 2000.0, 200000.0, 20000.0, 5000.0, 20000.0]),
                  np.array([4.0, -4.0, 0.0, 8.0, 4.0, 0.0]),
                  np.array([2.0, 2.0, 2.0, 2.0, 0.0, 8.0]))
# bins checked per point (widths 500, 1280 and 3463 fine points)
BINS = [0, 400, 1000]
TOL = {"fp64": 1e-9, "mixed": 1e-3}


@pytest.fixture(scope="module")
def full():
    return W.config(2)


@pytest.fixture(scope="module")
def reference(full):
    w = full
    ref = []
    for i in range(POINTS.n_points):
        steps, cnt, ex = oracle.odf_point(w.lines, w.species, w.species.abundance, float(POINTS.T_K[i]),
                                          float(POINTS.log10_P[i]), float(POINTS.vturb_kms[i]), w.layout,
                                          w.options, BINS)
        ref.append((steps, cnt, ambiguous_bins(ex["lq"], w.layout.bin_edges)))
    return ref


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_full_size_sampled_parity(full, reference, prec):
    import torch
    from paper_2105_13611_amd import odf
    w = full
    with odf.plan_for(w, precision=prec, workspace_bytes=WORKSPACE) as plan:
        out, st = plan.compute(w.species.abundance, POINTS)
        got = out.double().cpu().numpy()
    torch.cuda.synchronize()
    worst, worst_log, skipped = 0.0, 0.0, 0
    for i, (steps, cnt, amb) in enumerate(reference):
        for k, b in enumerate(BINS):
            if b in amb:
                skipped += 1
                continue
            worst = max(worst, float(rel_err(got[i, b], steps[k]).max()))
            worst_log = max(worst_log, float(log10_err(got[i, b], steps[k]).max()))
    n_surv = sum(c["survivors"] for _, c, _ in reference)
    n_samp = sum(c["voigt_samples"] for _, c, _ in reference)
    print(f"full size {prec}: max rel err per step {worst:.3e}, max |dlog10 k| {worst_log:.3e}, "
          f"skipped {skipped}; survivors {st['survivors']} (oracle {n_surv}), samples {st['voigt_samples']} "
          f"(oracle {n_samp})")
    assert skipped <= 2
    assert worst <= TOL[prec]
    assert abs(st["survivors"] - n_surv) <= 6
    assert abs(st["voigt_samples"] - n_samp) <= 6 * 2
    assert np.all(np.isfinite(got)) and np.all(got > 0)
    # monotone steps in every bin of every point (any size property)
    assert np.all(np.diff(got, axis=2) >= -1e-6 * np.abs(got[:, :, 1:]))

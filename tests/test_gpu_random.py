"""Randomised end-to-end parity: seeded small workloads with random options
(cutoff, window cap, mean, sub-bin fractions, electron pressure mode, bin
layout, wavelength interval, points), both precisions, against the oracle."""
from dataclasses import replace

import numpy as np
import pytest

from paper_2105_13611_amd import workload as W
from tests.gpu_helpers import compare_points

pytestmark = pytest.mark.gpu

TOL_STEP = {"fp64": 1e-9, "mixed": 1e-3}


@pytest.fixture(scope="module")
def odf():
    import torch
    assert torch.cuda.is_available()
    from paper_2105_13611_amd import odf as o
    o.load_library()
    return o


def random_workload(seed):
    rng = np.random.default_rng(1000 + seed)
    lo = 300.0 + rng.uniform(0.0, 6.0)
    hi = lo + rng.uniform(0.5, 4.0)
    n_lines = int(rng.integers(300, 3000))
    n_bins = int(rng.integers(1, 8))
    w = W.config(1, n_lines=n_lines, lam_range=(lo, hi), n_bins=n_bins)
    n_steps = int(rng.integers(1, 13))
    frac = rng.dirichlet(np.ones(n_steps))
    frac = frac / frac.sum()
    opts = replace(w.options, cutoff=float(rng.choice([1e-5, 1e-4, 1e-3])),
                   window_cap_doppler=float(rng.choice([50.0, 200.0, 500.0])),
                   mean=str(rng.choice(["geometric", "arithmetic"])),
                   electrons=str(rng.choice(["fixed", "equilibrium"])))
    n_pts = int(rng.integers(1, 4))
    pts = W.small_points(10.0 ** rng.uniform(np.log10(2500.0), np.log10(50000.0), n_pts),
                         rng.uniform(-2.0, 7.0, n_pts), rng.uniform(0.0, 8.0, n_pts))
    return replace(w, layout=replace(w.layout, step_frac=frac), options=opts, points=pts)


@pytest.mark.parametrize("seed", range(16))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_random_workload_parity(odf, seed, prec):
    w = random_workload(seed)
    with odf.plan_for(w, precision=prec, workspace_bytes=64 << 20) as plan:
        out, st = plan.compute(w.species.abundance, w.points)
        out = out.double().cpu().numpy()
        worst, worst_log, resolved = compare_points(w, out, prec, plan=plan)
    o = w.options
    print(f"seed {seed} {prec}: {w.lines.n_lines} lines, {w.layout.n_bins} bins x {w.layout.n_steps} steps, "
          f"cutoff {o.cutoff:g}, cap {o.window_cap_doppler:g}, {o.mean}, {o.electrons}, "
          f"{w.points.n_points} points: max rel err {worst:.3e}, near-tie bins {resolved}")
    assert worst <= TOL_STEP[prec]

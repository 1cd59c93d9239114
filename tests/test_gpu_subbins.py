"""Few-step ODFs (Sec. 4.1: two to four optimised sub-bins instead of the
standard twelve) through the HIP path, against the oracle, for both means."""
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


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("mean", ["geometric", "arithmetic"])
@pytest.mark.parametrize("fr", [(0.9, 0.1), (0.8, 0.15, 0.05), (0.5, 0.35, 0.13, 0.02)])
def test_few_step_odf_parity(odf, prec, mean, fr):
    w = W.config(1)
    w = replace(w, layout=replace(w.layout, step_frac=np.array(fr)),
                options=replace(w.options, mean=mean),
                points=W.small_points([5000.0, 3800.0], [4.0, 6.5], [2.0, 1.0]))
    with odf.plan_for(w, precision=prec, workspace_bytes=128 << 20) as plan:
        out, _ = plan.compute(w.species.abundance, w.points)
        assert tuple(out.shape) == (2, w.layout.n_bins, len(fr))
        out = out.double().cpu().numpy()
        worst, worst_log, resolved = compare_points(w, out, prec, plan=plan)
    print(f"{len(fr)} steps {mean} {prec}: max rel err {worst:.3e}, near-tie bins {resolved}")
    assert worst <= TOL_STEP[prec]

"""The allocation-free ODF reduction (odf_reduce_noalloc) against the
existing one (odf_stage_reduce) through the C ABI: same floor, sort and
sub-bin means, with the oversize-bin sort slabs in the library's static
device array instead of the workspace.  Layouts with bins beyond the LDS
capacity (20 000 and 42 576 points) make both paths use their global slab;
two calls in a row, the second with fewer grids, must each match the
existing entry point bit for bit."""
import numpy as np
import pytest

from paper_2105_13611_amd import workload as W

pytestmark = pytest.mark.gpu


def _workload(prec):
    N = W.grid_size(300.0, 340.0, W.RESOLVING_POWER)
    edges = np.array([0, 1, 4, 20004, N], dtype=np.int64)
    w = W.config(1, n_lines=50, lam_range=(300.0, 340.0))
    from dataclasses import replace
    lay = replace(w.layout, bin_edges=edges)
    return replace(w, layout=lay, options=replace(w.options, precision=prec)), N


def _grids(torch, n, N, dtype, seed):
    g = torch.Generator().manual_seed(seed)
    # log-uniform over 1e-7..1e3: much of it below the floor of about 2e-5
    x = torch.rand((n, N), generator=g, dtype=torch.float64) * 10.0 - 7.0
    return (10.0 ** x).to(dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_matches_stage_reduce(prec):
    import torch
    from paper_2105_13611_amd import odf
    w, N = _workload(prec)
    with odf.plan_for(w, workspace_bytes=64 << 20) as plan:
        print(f"[no-alloc] {prec}: N={N}, bins {np.diff(w.layout.bin_edges).tolist()}, "
              f"scratch per grid {plan.noalloc_scratch_need(1)} B", flush=True)
        assert plan.noalloc_scratch_need(1) > 0        # the static slab is used
        for call, n in enumerate((3, 1)):
            kap = _grids(torch, n, N, plan.out_dtype, 100 + call)
            out = torch.full((n, plan.n_bins, plan.n_steps), float("nan"), dtype=plan.out_dtype, device="cuda")
            plan.reduce_noalloc(kap, out)
            torch.cuda.synchronize()
            for i in range(n):
                ref = plan.stage_reduce(kap[i])
                torch.cuda.synchronize()
                assert torch.equal(out[i], ref), f"call {call}, grid {i}: differs from odf_stage_reduce"
            o = out.double().cpu().numpy()
            # monotone steps up to rounding (a one-point bin's steps are its
            # value, each rounded through its own log-mean)
            tol = 1e-12 if prec == "fp64" else 1e-6
            assert np.all(np.isfinite(o)) and np.all(np.diff(o, axis=2) >= -tol * np.abs(o[:, :, 1:]))


def test_noalloc_rejects_beyond_the_static_scratch():
    import ctypes as C
    import torch
    from paper_2105_13611_amd import odf
    w, N = _workload("fp64")
    with odf.plan_for(w, workspace_bytes=64 << 20) as plan:
        per = plan.noalloc_scratch_need(1)
        n_max = (32 << 20) // per
        n = n_max + 1
        kap = torch.ones((n, N), dtype=torch.float64, device="cuda")
        out = torch.empty((n, plan.n_bins, plan.n_steps), dtype=torch.float64, device="cuda")
        with pytest.raises(odf.OdfError) as e:
            plan.reduce_noalloc(kap, out)
        assert e.value.code == odf.ODF_E_NOMEM and "static scratch" in str(e.value)
        rc = odf.lib().odf_reduce_noalloc(plan.handle, None, 1, C.c_void_p(out.data_ptr()), None)
        assert rc == odf.ODF_E_INVALID
        # the largest count that fits still runs
        plan.reduce_noalloc(kap[:n_max].contiguous(), out[:n_max])
        torch.cuda.synchronize()
        assert torch.isfinite(out[:n_max]).all()

"""Request loop: continuous batching over a resident line list.

Requests with different compositions and point sets are submitted together;
each result must be bit-identical to the same request computed alone, the
requests must overlap on the device, a failed batch must fail only its own
ticket, and malformed or unknown tickets are rejected.
"""
from dataclasses import replace

import numpy as np
import pytest

from paper_2105_13611_amd import workload as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def odf():
    import torch
    assert torch.cuda.is_available()
    from paper_2105_13611_amd import odf as o
    o.load_library()
    return o


@pytest.fixture(scope="module")
def served():
    """A shrunk serving workload: shared line list and bins, per-request
    composition ([M/H], [alpha/Fe]) and T-P subsets."""
    w = W.config(4, n_lines=20_000, lam_range=(300.0, 345.0), n_bins=7, n_requests=6)
    rng = np.random.default_rng(44)
    reqs = []
    for r in w.requests:
        k = int(rng.integers(3, 19))
        idx = np.sort(rng.choice(r.points.n_points, k, replace=False))
        reqs.append(W.Request(r.abundance, r.points.take(idx), r.arrival_s))
    return replace(w, requests=reqs)


def _plan(odf, w, slots_points=4, n_slots=3):
    probe = odf.plan_for(w, workspace_bytes=256 << 20, max_batch_points=slots_points)
    ws = probe.request_footprint(slots_points) * n_slots + (1 << 20)
    probe.destroy()
    return odf.plan_for(w, workspace_bytes=ws, max_batch_points=slots_points, loop_streams=2)


def test_mix_equals_alone_and_overlaps(odf, served):
    w = served
    with _plan(odf, w) as plan:
        alone = [plan.compute(r.abundance, r.points)[0].clone() for r in w.requests]
        tickets = [plan.submit(r.abundance, r.points) for r in w.requests]
        stats = [plan.wait(t, 300.0) for t, _ in tickets]
        for (t, out), a, st, r in zip(tickets, alone, stats, w.requests):
            assert st["state"] == "DONE", st
            assert st["points"] == r.points.n_points
            assert st["line_evals"] == r.points.n_points * w.lines.n_lines
            assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
            assert bool((out == a).all()), "result differs between alone and in the mix"
        # continuous batching: some request was admitted while another was still running
        overlap = any(stats[j]["t_admit"] < stats[i]["t_done"] and stats[i]["t_admit"] < stats[j]["t_done"]
                      for i in range(len(stats)) for j in range(len(stats)) if i != j)
        assert overlap


def test_failed_batch_fails_only_its_ticket(odf, served):
    w = served
    big = W.Points(np.tile(w.requests[1].points.T_K, 8), np.tile(w.requests[1].points.log10_P, 8),
                   np.tile(w.requests[1].points.vturb_kms, 8))
    with _plan(odf, w) as plan:
        ref0 = plan.compute(w.requests[0].abundance, w.requests[0].points)[0].clone()
        ref2 = plan.compute(w.requests[2].abundance, w.requests[2].points)[0].clone()
        t0, o0 = plan.submit(w.requests[0].abundance, w.requests[0].points)
        t1, o1 = plan.submit(w.requests[1].abundance, big)
        plan.fail_next_batch(t1)
        t2, o2 = plan.submit(w.requests[2].abundance, w.requests[2].points)
        s0, s1, s2 = plan.wait(t0), plan.wait(t1), plan.wait(t2)
        assert s1["state"] == "FAILED" and "forced failure" in s1["msg"]
        assert s0["state"] == "DONE" and s2["state"] == "DONE"
        assert bool((o0 == ref0).all()) and bool((o2 == ref2).all())


def test_unknown_ticket_invalid_request_and_empty_request(odf, served):
    w = served
    with _plan(odf, w) as plan:
        with pytest.raises(odf.OdfError) as e:
            plan.poll(987654)
        assert e.value.code == odf.ODF_E_UNKNOWN_TICKET
        bad = W.Points(np.array([-5.0]), np.array([1.0]), np.array([2.0]))
        with pytest.raises(odf.OdfError) as e:
            plan.submit(w.species.abundance, bad)
        assert e.value.code == odf.ODF_E_INVALID
        empty = W.Points(np.zeros(0), np.zeros(0), np.zeros(0))
        t, _ = plan.submit(w.species.abundance, empty)
        assert plan.wait(t, 30.0)["state"] == "DONE"


def test_footprint_and_admission_bound(odf, served):
    w = served
    with _plan(odf, w) as plan:
        f1, f4, f100 = plan.request_footprint(1), plan.request_footprint(4), plan.request_footprint(100)
        assert 0 < f1 <= f4 <= f100 <= plan.workspace.numel()
        # more requests than slots: all complete, in any order, each exactly once
        tickets = [plan.submit(r.abundance, r.points) for r in w.requests * 2]
        for t, _ in tickets:
            assert plan.wait(t, 300.0)["state"] == "DONE"


def test_compute_waits_for_the_loop(odf, served):
    w = served
    with _plan(odf, w) as plan:
        ref = plan.compute(w.requests[3].abundance, w.requests[3].points)[0].clone()
        tickets = [plan.submit(r.abundance, r.points) for r in w.requests]
        # a blocking compute while the loop is busy takes the workspace in turn
        again = plan.compute(w.requests[3].abundance, w.requests[3].points)[0]
        assert bool((again == ref).all())
        for t, _ in tickets:
            assert plan.wait(t, 300.0)["state"] == "DONE"

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


def _plan(odf, w, slots_points=4, n_slots=5):
    """A plan whose pool holds n_slots batch slots of slots_points points
    (a request of more than that many points reserves two of them)."""
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
    """Admission by footprint: a request reserves min(n, 4)-point slots, two
    of them once it has more than one batch; the pool holds five 4-point
    slots, so small requests are resident together while large ones wait
    for room.  Sampled while the loop runs, the reserved bytes never exceed
    the pool, and every result equals the request computed alone."""
    import time
    import torch
    w = served
    with _plan(odf, w) as plan:
        st0 = plan.loop_status()
        f0, f1, f3, f4, f5, f100 = (plan.request_footprint(n) for n in (0, 1, 3, 4, 5, 100))
        assert f0 == 0 and 0 < f1 < f3 < f4 and f5 == f100 == 2 * f4
        assert st0["slot_points"] == 4 and st0["slots_per_request"] == 2
        pool = st0["pool_bytes"]
        assert 5 * f4 <= pool < 6 * f4 and pool <= plan.workspace.numel()
        # requests of 1..18 points, more than fit at once
        rng = np.random.default_rng(3)
        reqs = []
        for k in range(14):
            r = w.requests[k % len(w.requests)]
            n = int(rng.integers(1, min(18, r.points.n_points) + 1))
            reqs.append(W.Request(r.abundance, r.points.take(np.arange(n)), 0.0))
        alone = [plan.compute(r.abundance, r.points)[0].clone() for r in reqs]
        tickets = [plan.submit(r.abundance, r.points) for r in reqs]
        seen = []
        while True:
            st = plan.loop_status()
            seen.append(st)
            assert st["resident_bytes"] <= pool and st["peak_resident_bytes"] <= pool
            if all(plan.poll(t)["state"] in ("DONE", "FAILED") for t, _ in tickets):
                break
            time.sleep(0.002)
        torch.cuda.synchronize()
        stats = [plan.wait(t, 60.0) for t, _ in tickets]
        for st, (t, out), a, r in zip(stats, tickets, alone, reqs):
            assert st["state"] == "DONE", st
            assert bool((out == a).all())
        end = plan.loop_status()
    assert end["resident_bytes"] == 0 and end["resident_requests"] == 0 and end["batches_in_flight"] == 0
    assert 2 <= end["peak_resident_requests"] and end["peak_resident_bytes"] <= pool
    assert max(s["queued_requests"] for s in seen) > 0       # some waited for room
    # arrival order: a request is never admitted before an earlier one
    admits = [s["t_admit"] for s in stats]
    assert all(admits[i] <= admits[i + 1] for i in range(len(admits) - 1))
    print(f"pool {pool} B ({pool / f4:.2f} slots of 4 points): peak {end['peak_resident_bytes']} B, "
          f"{end['peak_resident_requests']} requests resident at most, "
          f"{max(s['queued_requests'] for s in seen)} queued at most")


def test_submit_orders_after_the_callers_stream(odf, served):
    """A request's device work starts only after what was queued on the
    plan's stream before submit: here a long chain of products and then a
    fill of the output buffer with NaN; the result must be the request's,
    not the fill."""
    import torch
    w = served
    r = w.requests[2]
    with _plan(odf, w) as plan:
        ref = plan.compute(r.abundance, r.points)[0].clone()
        out = plan.new_out(r.points.n_points)
        a = torch.randn(4096, 4096, device=plan.device)
        with torch.cuda.stream(plan.stream):
            for _ in range(40):
                a = (a @ a).div_(a.abs().max())
            out.fill_(float("nan"))
        t, _ = plan.submit(r.abundance, r.points, out)
        st = plan.wait(t, 300.0)
        torch.cuda.synchronize()
    assert st["state"] == "DONE"
    assert bool((out == ref).all())


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

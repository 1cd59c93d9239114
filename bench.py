"""ODF-generation benchmark on one MI355X.

Workload: the full DFSYNTHE-style table (57 temperatures x 25 pressures at
v_turb = 2 km/s, 1e7 synthetic lines from 9 nm to 10 um over 40 species x 2
stages, R = 500 000 grid of 3 507 864 points, 1212 ramp bins, 12 sub-bins).
A step is one odf_compute over the whole table; the inputs (line list,
composition, point list) are resident or in host memory before timing, the
output stays in device memory.  Both precisions are timed: the FP32
compensated ("mixed") path is the headline value, the plain FP64 path is
reported beside it.

Roofline of the dominant kernel (the Voigt scatter-sum) is measured live with
HIP events the library records around every launch on its stream; the rate
uses the union of the launch intervals (the two internal streams overlap
launches), and the HBM traffic comes from the committed counter summary
while the kernel sources still match it.
The CPU baseline times the FP64 oracle on a bounded stratified sample of the
same workload and scales it to points/s.  It runs first, before anything
touches the GPU, and its oracle ODF steps are kept: the line's "parity" block
compares both GPU paths with them at the sampled (point, bin) pairs.

The headline mixed leg runs the given --steps/--warmup; the plain FP64 leg,
about six times slower per table, runs its own bounded count (--fp64-steps,
--fp64-warmup; 2 and 1 by default), stated in the line.

--mode pretab times the pre-tabulated high-resolution opacity of a
wavelength interval (one value per fine point) over the same T-P table and
reports the T-P interpolation error of that opacity; --mode subbins searches
2-4-sub-bin ODF configurations against the standard 12 with an isothermal
slab as the consumer; --mode serve runs a request stream.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--mode table|pretab|serve]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ODF (T,P) points/s + line evals/s, FP32 vs FP64 plain at ≤1e-3 ODF err"

WORKLOADS = {
    2: ("DFSYNTHE-style table: 57 T x 25 log P at vturb 2 km/s, 1e7 synthetic lines 9 nm-10 um "
        "(40 species x 2 stages), R=5e5 grid of 3507864 points, 1212 ramp bins x 12 sub-bins"),
    3: ("DFSYNTHE-style table at five microturbulences: 57 T x 25 log P x vturb {0,1,2,4,8} km/s "
        "(7125 points), 1e7 synthetic lines 9 nm-10 um (40 species x 2 stages), R=5e5 grid of "
        "3507864 points, 1212 ramp bins x 12 sub-bins"),
    5: ("large line list: 57 T x 25 log P x vturb {0,1,2,4,8} km/s (7125 points), 1e8 synthetic lines "
        "9 nm-10 um (80 species x 3 stages), R=5e5 grid of 3507864 points, 1212 ramp bins x 12 sub-bins"),
}

# nominal FP32 operations per Voigt sample on the far-wing path (the path
# almost every sample takes), FMA = 2: u carried from the previous row 2,
# u from the index at the first of eight rows 6/8, v = u^2 + D 2, numerator
# 2, denominator 2, reciprocal 1, accumulate 2, compensated add every 64
# lines 4/64
FLOP_PER_SAMPLE_F32 = 11.8
# FP64 far wing (four-node pair as one fraction in X = x^2): x carried 2,
# X 1, numerator and denominator Horner chains 14, reciprocal with one Newton
# step 5, product and accumulate 3, edge mask 3
FLOP_PER_SAMPLE_F64 = 28
# VALU rate without packed FP32 (disabled in this build): 256 CU x 4 SIMD x
# 16 lanes x 2 FLOP per FMA x 2.4 GHz, a ceiling reported beside the
# published peaks
PEAK_VALU_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
# published MI355X vector peaks: FP32 (with packed FP32 instructions) and FP64
PEAK_F32_DATASHEET = 157.3
PEAK_F64_DATASHEET = 78.6
# parity tolerances per ODF step (relative): mixed path and plain FP64 path
TOL = {"mixed": 1e-3, "fp64": 1e-9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def stratified_points(points, n, seed=2):
    """The four T-P corners, (5000 K, log P = 4) and seeded random points."""
    import numpy as np
    T, P = points.T_K, points.log10_P
    idx = []
    for t, p in [(T.min(), P.min()), (T.min(), P.max()), (T.max(), P.min()), (T.max(), P.max())]:
        idx.append(int(np.argmin(np.abs(np.log(T / t)) + np.abs(P - p))))
    idx.append(int(np.argmin(np.abs(np.log(T / 5000.0)) + np.abs(P - 4.0))))
    rng = np.random.default_rng(seed)
    rest = [i for i in rng.permutation(points.n_points) if i not in idx]
    idx += rest[: max(0, n - len(idx))]
    return np.array(sorted(set(idx[:n])), dtype=np.int64)


def run_gpu(w, precision, steps, warmup, workspace_gb, points_idx=None, batch_points=0, sample=None,
            alone=True):
    """One leg: plan, `warmup` untimed steps, `steps` timed steps over the
    table (or its stratified subset).  sample = (point indices into
    w.points, bins): the output at those pairs is returned for the parity
    block (points outside this leg's subset are left out).  alone: also time
    the Voigt kernel by itself on 72 stratified points (after the timed
    steps; a profiled run leaves it out so that its counters cover the
    table's launches only)."""
    import numpy as np
    import torch
    from paper_2105_13611_amd import odf
    pts = w.points if points_idx is None else w.points.take(points_idx)
    t0 = time.perf_counter()
    plan = odf.plan_for(w, precision=precision, workspace_bytes=int(workspace_gb * (1 << 30)),
                        kernel_timing=True, max_batch_points=batch_points)
    t_plan = time.perf_counter() - t0
    out = plan.new_out(pts.n_points)
    for k in range(warmup):
        log(f"[bench] {precision}: warmup step {k + 1}/{warmup}")
        plan.compute(w.species.abundance, pts, out)
    plan.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for k in range(steps):
        _, stats = plan.compute(w.species.abundance, pts, out)
        log(f"[bench] {precision}: step {k + 1}/{steps} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = plan.stage_times(reset=True)
    res = dict(precision=precision, seconds=dt, steps=steps, warmup=warmup, n_points=pts.n_points,
               plan_seconds=t_plan, stats=stats, stage_ms=times,
               batch_points=None, checksum=float(out.double().sum().item()))
    if sample is not None:
        where = (np.arange(w.points.n_points) if points_idx is None else np.asarray(points_idx))
        row = {int(g): k for k, g in enumerate(where)}
        got = {}
        for i in sample[0]:
            if int(i) in row:
                got[int(i)] = out[row[int(i)]][list(sample[1])].double().cpu().numpy()
        res["sample_out"] = got
    if alone:
        res["kernel_alone"] = kernel_alone(plan, w)
    plan.destroy()
    del out
    torch.cuda.empty_cache()
    return res


def kernel_alone(plan, w, n_points=72, chunk=24):
    """The Voigt kernel with nothing beside it: requests of `chunk` points are
    one batch each, so preparation, Voigt and reduction run one after the
    other and each Voigt launch has the GPU to itself.  Stratified points of
    the table, outside the timed region."""
    pts = w.points.take(stratified_points(w.points, n_points))
    plan.stage_times(reset=True)
    samples = 0
    for i in range(0, pts.n_points, chunk):
        _, st = plan.compute(w.species.abundance, pts.take(slice(i, i + chunk)))
        samples += st["voigt_samples"]
    t = plan.stage_times(reset=True)["voigt"]
    return dict(ms=t["ms"], busy_ms=t["busy_ms"], launches=t["launches"], samples=samples,
                points=pts.n_points, batch_points=chunk)


def kernel_sources_sha256():
    """Hash of the sources that define the Voigt kernels: a traffic figure
    taken from counters applies only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("k_voigt.hip", "odf_internal.h"):
        with open(os.path.join(ROOT, "paper_2105_13611_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_per_launch(precision, samples_per_launch=None):
    """HBM bytes per Voigt launch from the committed counter summary of the
    full-table run (FETCH_SIZE + WRITE_SIZE, each scaled by its copy-kernel
    calibration), or None when there is none or the kernel has changed.
    Given this run's samples per launch, the summary's bytes per sample are
    scaled to it (the same table may be cut into launches differently)."""
    path = os.path.join(ROOT, "profiles", f"voigt{32 if precision == 'mixed' else 64}_full_table_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    i = txt.find("```json")
    if i < 0:
        return None
    d = json.loads(txt[i + 7: txt.index("```", i + 7)])
    if d.get("source_sha256") != kernel_sources_sha256():
        return None
    if samples_per_launch is not None and "hbm_bytes_per_sample" in d:
        return d["hbm_bytes_per_sample"] * samples_per_launch
    return d["hbm_bytes_per_launch"]


def executed_flop_per_sample(precision):
    """FP32 (mixed) or FP64 operations the Voigt kernel executed per Voigt
    sample, from the committed VALU-counter summary of the full-table run, or
    None when there is none or the kernel has changed since."""
    path = os.path.join(ROOT, "profiles", f"voigt{32 if precision == 'mixed' else 64}_full_table_valu_flops.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    i = txt.find("```json")
    if i < 0:
        return None
    d = json.loads(txt[i + 7: txt.index("```", i + 7)])
    if d.get("source_sha256") != kernel_sources_sha256():
        return None
    return d["executed_flop_per_sample"]


def roofline(res, flop_per_sample, precision):
    """Roofline of the Voigt kernel of one leg.  achieved = the method's
    FLOP per launch (Voigt samples per launch x nominal FLOP per sample) over
    the kernel's average launch duration (HIP events on the launch's stream,
    the figure rocprofv3's kernel trace reports); peak = the published vector
    peak of the path's type (FP32 157.3, FP64 78.6 TFLOP/s).  The two summing
    streams overlap launches, so a launch's duration includes time it shares
    the GPU; achieved_busy uses the union of the launch intervals instead.
    The mixed path also carries the non-packed FP32 rate (packed FP32 is
    disabled in this build) as a ceiling of its own."""
    st = res["stage_ms"]["voigt"]
    ms, busy, launches = st["ms"], st["busy_ms"], st["launches"]
    samples = res["stats"]["voigt_samples"] * res["steps"]
    if launches == 0 or busy <= 0 or ms <= 0:
        return None
    peak = PEAK_F32_DATASHEET if precision == "mixed" else PEAK_F64_DATASHEET
    flop_per_launch = samples * flop_per_sample / launches
    achieved = flop_per_launch / (ms / 1e3 / launches) / 1e12
    achieved_busy = flop_per_launch / (busy / 1e3 / launches) / 1e12
    out = dict(bound="alu", achieved=achieved, peak=peak, unit="TFLOP/s", frac=achieved / peak,
               traffic=traffic_per_launch(precision, samples / launches),
               kernel="k_voigt32" if precision == "mixed" else "k_voigt64",
               avg_launch_ms=ms / launches, busy_ms_per_launch=busy / launches, launches=launches,
               samples_per_launch=samples / launches, flop_per_sample=flop_per_sample,
               achieved_busy=achieved_busy, frac_busy=achieved_busy / peak)
    if precision == "mixed":
        out["ceiling_nonpacked"] = dict(peak=PEAK_VALU_TFLOPS, frac=achieved / PEAK_VALU_TFLOPS,
                                        note="256 CU x 4 SIMD x 16 lanes x 2 FLOP per FMA x 2.4 GHz: the "
                                             "FP32 rate without packed FP32 instructions")
        out["note"] = ("achieved counts every Voigt sample of the method (each (line, fine point) pair in "
                       "the windows) at the far-wing cost; lines whose window covers a 1024-point tile from "
                       "more than 64 (128, 384, 1536) points away are evaluated at 64 (32, 16, 8) nodes of "
                       "the tile and interpolated, so the kernel evaluates fewer samples: executed is what "
                       "its VALU did (counters)")
    e = executed_flop_per_sample(precision)
    if e is not None:
        xa = samples * e / (ms / 1e3) / 1e12
        out["executed"] = dict(flop_per_sample=e, achieved=xa, frac=xa / peak)
    ka = res.get("kernel_alone")
    if ka and ka["ms"] > 0:
        a = ka["samples"] * flop_per_sample / (ka["ms"] / 1e3) / 1e12
        out["kernel_alone"] = dict(achieved=a, frac=a / peak,
                                   avg_launch_ms=ka["ms"] / ka["launches"], launches=ka["launches"],
                                   points=ka["points"], batch_points=ka["batch_points"],
                                   note="same kernel with no other kernel beside it (requests of one batch "
                                        "each, so preparation, Voigt and reduction run in turn), stratified "
                                        "points, outside the timed region")
    return out


# bins of the CPU leg: 24 keep its oracle work near 30 s of wall time on 16
# cores (64 took 79 s); the GPU tests check 64-bin samples
CPU_BINS = 24


def cpu_sample(w):
    """The CPU leg's sample: 16 stratified points of the table and 24 bins
    evenly spaced over the layout (the first and the last included)."""
    import numpy as np
    nb = w.layout.n_bins
    k = min(CPU_BINS, nb)
    return stratified_points(w.points, 16), [int(b) for b in np.round(np.linspace(0, nb - 1, k))]


def cpu_baseline(w, workers):
    """Oracle throughput on a stratified sample of points and bins, scaled to
    points/s over the same table: per point, the line stage is timed in full
    and the Voigt sum on a few bins, extrapolated by the point's total sample
    count (which the oracle's line stage reports for the whole grid).  Runs
    before anything touches the GPU (the pool forks this process).  Returns
    the baseline and the oracle's ODF steps at the sampled (point, bin)
    pairs, for the parity block."""
    import multiprocessing as mp
    import numpy as np
    global _CPU_W
    idx, bins = cpu_sample(w)
    tasks = [(int(i), bins) for i in idx]
    # the forked workers inherit the workload; tasks carry only indices
    _CPU_W = w
    t0 = time.perf_counter()
    try:
        with mp.get_context("fork").Pool(min(workers, len(tasks))) as pool:
            per = pool.map(_cpu_task, tasks, chunksize=1)
    finally:
        _CPU_W = None
    wall = time.perf_counter() - t0
    core_s = [p["t_lines"] + p["t_bins"] * p["samples_total"] / max(p["samples_bins"], 1) for p in per]
    mean_core_s = float(np.mean(core_s))
    value = workers / mean_core_s
    base = dict(value=value, unit="points/s", cores=workers, kind="oracle",
                sample=(f"{len(idx)} stratified (T,P) points of the table x {len(bins)} bins evenly spaced "
                        f"over the {w.layout.n_bins} "
                        f"({sum(p['samples_bins'] for p in per)} Voigt samples, wall {wall:.1f} s on "
                        f"{min(workers, len(tasks))} processes); per point the line stage is timed in "
                        f"full and the bin sums are scaled by total/sampled Voigt samples; "
                        f"points/s = cores / mean core-seconds per point ({mean_core_s:.0f} s)"),
                wall_s=wall, mean_core_s_per_point=mean_core_s)
    ref = {p["point"]: dict(steps=p["steps"], near_tie=p["near_tie"]) for p in per}
    return base, ref, bins


def _near_tie_bins(lq, edges, bins):
    """Bins whose fine-grid opacity depends on a decision that floating
    point takes within rounding of its boundary (a keep test with
    |core/thr - 1| < 1e-11, or a window edge within 1e-7 of an integer):
    there either result is valid, so the parity block counts them."""
    import numpy as np
    with np.errstate(divide="ignore", invalid="ignore"):
        tie = np.abs(lq["core"] / lq["thr"] - 1.0) < 1e-11
    tie |= lq["keep"] & ((np.abs(lq["jlo_r"] - np.round(lq["jlo_r"])) < 1e-7)
                         | (np.abs(lq["jhi_r"] - np.round(lq["jhi_r"])) < 1e-7))
    out = []
    for b in bins:
        j0, j1 = int(edges[b]), int(edges[b + 1])
        out.append(bool(np.any(tie & (lq["jlo"] - 1 <= j1 - 1) & (lq["jhi"] + 1 >= j0))))
    return out


_CPU_W = None


def _cpu_task(args):
    import numpy as np
    import oracle
    w = _CPU_W
    i, bins = args
    T, lp, v = float(w.points.T_K[i]), float(w.points.log10_P[i]), float(w.points.vturb_kms[i])
    t0 = time.perf_counter()
    lq = oracle.line_quantities(w.lines, w.species, w.species.abundance, T, lp, v, w.layout, w.options)
    t_lines = time.perf_counter() - t0
    s = lq["surv"]
    total = int(np.sum(lq["jhi"][s] - lq["jlo"][s] + 1))
    e = w.layout.bin_edges
    nsb = 0
    steps = []
    t0 = time.perf_counter()
    for b in bins:
        j0, j1 = int(e[b]), int(e[b + 1])
        m = s & (lq["jlo"] <= j1 - 1) & (lq["jhi"] >= j0)
        nsb += int(np.sum(np.minimum(lq["jhi"][m], j1 - 1) - np.maximum(lq["jlo"][m], j0) + 1))
        kl = oracle.fine_opacity(lq, w.layout, j0, j1)
        fl = w.options.cutoff * oracle.physics.kappa_c(oracle.grid_lambda_nm(w.layout, np.arange(j0, j1)), w.options)
        steps.append(oracle.odf_reduce_bin(np.maximum(kl, fl), w.layout.step_frac, w.options.mean))
    t_bins = time.perf_counter() - t0
    return dict(point=i, t_lines=t_lines, t_bins=t_bins, samples_total=total, samples_bins=nsb,
                steps=np.stack(steps), near_tie=_near_tie_bins(lq, e, bins))


def parity_block(ref, bins, legs):
    """Max relative error per ODF step and max |dlog10 kappa| of each GPU
    leg against the oracle's steps at the CPU leg's sampled pairs."""
    import numpy as np
    out = dict(sample=f"{len(ref)} stratified (T,P) points x {len(bins)} bins evenly spaced of the timed table "
                      f"(first {bins[0]}, last {bins[-1]}), oracle steps from the CPU leg", tolerance=dict(TOL))
    for prec, got in legs.items():
        rel, dlog, pairs, ties, worst_tie = 0.0, 0.0, 0, 0, 0.0
        for i, r in ref.items():
            if i not in got:
                continue
            for k in range(len(bins)):
                g, o = got[i][k], r["steps"][k]
                e = float(np.max(np.abs(g / o - 1.0)))
                pairs += 1
                if r["near_tie"][k]:
                    ties += 1
                    worst_tie = max(worst_tie, e)
                rel = max(rel, e)
                dlog = max(dlog, float(np.max(np.abs(np.log10(g) - np.log10(o)))))
        out[prec] = dict(max_rel_err=rel, max_abs_dlog10_kappa=dlog, pairs=pairs,
                         within_tolerance=bool(pairs > 0 and rel <= TOL[prec]),
                         bins_with_near_tie_decisions=ties, max_rel_err_in_those=worst_tie)
    return out


def run_serving(n_requests, rate_hz, workspace_gb, max_points, serve_config=4):
    """Continuous-batching run on a request stream over a shared resident line
    list and bins (mixed precision).  Stream 4: Poisson arrivals (20 req/s
    unless rate_hz), each request with its own composition ([M/H],
    [alpha/Fe]) and a random subset of the 1425 T-P points, 1e7 lines.
    Stream 5: bursts of 8 requests (5 req/s mean), each the whole grid at five
    vturb, 1e8 lines over 80 species x 3 stages.  Requests are submitted at
    their arrival times; latency is t_done - t_submit."""
    import numpy as np
    import torch
    from paper_2105_13611_amd import odf
    from paper_2105_13611_amd import workload as W
    w = W.config(serve_config, n_requests=n_requests)
    reqs = w.requests
    if rate_hz and serve_config == 4:
        reqs = W.draw_requests_cfg4(4, w.species, w.points, n_requests, rate_hz=rate_hz)
    if max_points:
        # evenly spaced over each request's point list (the list runs through
        # the grid in order, so a prefix would keep only its cheapest end)
        reqs = [W.Request(r.abundance, r.points.take(np.unique(np.linspace(
                    0, r.points.n_points - 1, min(max_points, r.points.n_points)).astype(np.int64))),
                          r.arrival_s) for r in reqs]
    plan = odf.plan_for(w, precision="mixed", workspace_bytes=int(workspace_gb * (1 << 30)))
    outs = [plan.new_out(r.points.n_points) for r in reqs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = []
    for r, o in zip(reqs, outs):
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append((plan.submit(r.abundance, r.points, o)[0], time.perf_counter()))
    stats = []
    for (t, t_sub), r in zip(tickets, reqs):
        st = plan.wait(t, 3600.0)
        stats.append(st)
        log(f"[serve] request {t}: {r.points.n_points} points, {st['state']}, "
            f"latency {st['t_done'] - st['t_submit']:.2f} s")
    wall = time.perf_counter() - t0
    lat = np.array([s["t_done"] - s["t_submit"] for s in stats])
    wait = np.array([s["t_admit"] - s["t_submit"] for s in stats])
    pts = sum(r.points.n_points for r in reqs)
    span = max(s["t_done"] for s in stats) - min(s["t_submit"] for s in stats)
    res = dict(metric="ODF serving: latency percentiles and points/s under a request stream",
               mode="serve", stream=serve_config, requests=len(reqs),
               rate_hz=rate_hz or (20.0 if serve_config == 4 else 5.0),
               offered_points_per_s=pts / max(reqs[-1].arrival_s, 1e-9),
               achieved_points_per_s=pts / span, wall_s=wall,
               # compositions differ per request ([M/H] mostly below solar: fewer
               # and narrower surviving lines), so the work per point differs from
               # the table's; samples/s compares across streams
               achieved_voigt_samples_per_s=sum(s["voigt_samples"] for s in stats) / span,
               achieved_line_evals_per_s=sum(s["line_evals"] for s in stats) / span,
               latency_s=dict(p50=float(np.percentile(lat, 50)), p95=float(np.percentile(lat, 95)),
                              p99=float(np.percentile(lat, 99)), max=float(lat.max())),
               admission_wait_s=dict(p50=float(np.percentile(wait, 50)), max=float(wait.max())),
               points=pts, failed=sum(s["state"] != "DONE" for s in stats),
               slots=None, dtype="f32", data="synthetic",
               config={"workload": ("serving stream over the 1e7-line table: per-request composition "
                                    "and 1..1425 T-P points at vturb 2 km/s, 1212 bins x 12 sub-bins"
                                    if serve_config == 4 else
                                    "serving stream over the 1e8-line list (80 species x 3 stages): bursts "
                                    "of 8 requests, each the 7125-point grid at five vturb, 1212 bins x 12 "
                                    "sub-bins")
                                   + (f" [each request cut to {max_points} evenly spaced points]" if max_points else "")})
    plan.destroy()
    return res


PRETAB_METRIC = "pre-tabulated high-resolution opacity: (T,P) points/s"


def _lattice(lt, lp):
    """Points of a log10 T x log10 P lattice, P fastest."""
    from paper_2105_13611_amd import workload as W
    import numpy as np
    TT, PP = np.meshgrid(10.0 ** np.asarray(lt), np.asarray(lp), indexing="ij")
    return W.Points(TT.ravel(), PP.ravel(), np.full(TT.size, 2.0))


def interpolation_study(plan, w, T_range=(4000.0, 12000.0), P_range=(0.0, 6.0), refine=(1, 2)):
    """T-P interpolation error of the pre-tabulated opacity (Sec. 4.1; the
    T-P grid of Sec. 4.2).  A lattice with the DFSYNTHE steps (log10 T by
    2/56, log10 P by 0.5), and the same refined, over a sub-range of the
    table: the opacity computed at the centre of every cell against the
    bilinear interpolation in (log T, log P) of log kappa from its four
    corners, over every fine point."""
    import numpy as np
    import torch
    out = {}
    for r in refine:
        dT, dP = (2.0 / 56.0) / r, 0.5 / r
        k0 = math.floor(math.log10(T_range[0] / 2000.0) / (2.0 / 56.0))
        lt = math.log10(2000.0) + k0 * (2.0 / 56.0) + dT * np.arange(
            int(math.ceil((math.log10(T_range[1]) - math.log10(2000.0) - k0 * 2.0 / 56.0) / dT)) + 1)
        lp = P_range[0] + dP * np.arange(int(round((P_range[1] - P_range[0]) / dP)) + 1)
        nodes = _lattice(lt, lp)
        cent = _lattice(0.5 * (lt[:-1] + lt[1:]), 0.5 * (lp[:-1] + lp[1:]))
        t0 = time.perf_counter()
        kn, _ = plan.compute(w.species.abundance, nodes)
        kc, _ = plan.compute(w.species.abundance, cent)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ln = kn.double().log().view(lt.size, lp.size, -1)
        li = 0.25 * (ln[:-1, :-1] + ln[1:, :-1] + ln[:-1, 1:] + ln[1:, 1:])
        err = (li.reshape(kc.shape) - kc.double().log()).exp().sub(1.0).abs()
        sub = err[:, ::16].flatten().cpu().numpy()
        out[f"step_1/{r}"] = dict(
            log10_T_step=dT, log10_P_step=dP, nodes=nodes.n_points, centres=cent.n_points,
            median=float(np.median(sub)), p99=float(np.percentile(sub, 99.0)),
            max=float(err.max().item()), frac_above_1pct=float((err > 0.01).double().mean().item()),
            frac_above_3pct=float((err > 0.03).double().mean().item()), seconds=dt)
        log(f"[bench] interpolation at 1/{r} of the DFSYNTHE steps: {out[f'step_1/{r}']}")
        del kn, kc, ln, li, err
        torch.cuda.empty_cache()
    out["T_range_K"] = list(T_range)
    out["log10_P_range"] = list(P_range)
    out["note"] = ("relative error of exp(bilinear interpolation of ln kappa in (log T, log P)) at cell "
                   "centres against the computed floored opacity; median and p99 over every 16th fine "
                   "point, max and fractions over all")
    return out


def run_pretab(args):
    """Pre-tabulated high-resolution opacity (Sec. 4.1): the floored line
    opacity of every fine point of a wavelength interval at R = 5e5, over
    the DFSYNTHE T-P table, and the T-P interpolation study."""
    import numpy as np
    import torch
    from dataclasses import replace
    from paper_2105_13611_amd import odf
    from paper_2105_13611_amd import workload as W
    lo, hi = args.pretab_nm
    # the full list's line density (1e7 lines log-uniform over 9 nm - 10 um)
    n_lines = int(round(1e7 * math.log(hi / lo) / math.log(W.LAMBDA_LAST_FULL_NM / 9.0)))
    w = W.config(2, n_lines=n_lines, lam_range=(lo, hi), n_bins=1)
    w = replace(w, options=replace(w.options, output="fine"))
    N = W.grid_size(lo, hi, W.RESOLVING_POWER)
    prec = "mixed" if args.precision == "both" else args.precision
    log(f"[bench] pretab: {n_lines} lines in {lo}-{hi} nm, N = {N}, {w.points.n_points} points, {prec}")
    plan = odf.plan_for(w, precision=prec, workspace_bytes=int(args.workspace_gb * (1 << 30)),
                        kernel_timing=True)
    out = plan.new_out(w.points.n_points)
    for k in range(args.warmup):
        plan.compute(w.species.abundance, w.points, out)
    plan.stage_times(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = None
    for k in range(args.steps):
        _, stats = plan.compute(w.species.abundance, w.points, out)
        log(f"[bench] pretab: step {k + 1}/{args.steps} done at {time.perf_counter() - t0:.2f} s")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    times = plan.stage_times(reset=True)
    value = w.points.n_points * args.steps / dt
    fine = times["odf"]
    # the fine-output kernel: one read and one write per fine point
    bytes_per_launch = (8 if prec == "fp64" else 4) * 2 * N * w.points.n_points * args.steps / max(fine["launches"], 1)
    res = {
        "metric": PRETAB_METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": dt / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"pre-tabulated opacity {lo}-{hi} nm at R=5e5 ({N} fine points), "
                               f"{n_lines} synthetic lines (the 1e7-line list's density), "
                               f"57 T x 25 log P at vturb 2 km/s",
                   "points": w.points.n_points, "lines": n_lines, "grid_points": N},
        "fine_points_per_s": value * N,
        "voigt_samples_per_s": stats["voigt_samples"] * args.steps / dt,
        "stage_ms": {k: v["ms"] for k, v in times.items()},
        "stage_busy_ms": {k: v["busy_ms"] for k, v in times.items()},
        "fine_output_kernel": dict(launches=fine["launches"], avg_launch_ms=fine["ms"] / max(fine["launches"], 1),
                                   achieved_GBs=bytes_per_launch / (fine["ms"] / max(fine["launches"], 1)) / 1e6,
                                   peak_GBs=8000.0),
        "checksum": float(out.double().sum().item()),
    }
    del out
    torch.cuda.empty_cache()
    if not args.no_interp:
        res["interpolation"] = interpolation_study(plan, w)
    plan.destroy()
    return res


SUBBIN_METRIC = "ODF error of an isothermal slab, |I_ODF/I_N - 1| over points, bins and columns"
# slab columns as continuum optical depths kappa_c m at the bin centre: the
# lines matter while the continuum is thin (a slab thick in the continuum
# radiates the Planck function whatever the lines)
SLAB_TAU_C = (1e-4, 1e-3, 1e-2, 0.1, 1.0)
BORDER_CANDIDATES = (0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.75, 0.8, 0.85, 0.9, 0.925, 0.95, 0.965, 0.975,
                     0.985, 0.99, 0.995)
N_ELEMENTARY = 200


def combine_steps(elem, borders, mean, n_elem=N_ELEMENTARY):
    """Sub-bin means of a configuration from an ODF of n_elem equal
    elementary sub-bins: borders are cumulative fractions (multiples of
    1/n_elem, without 0 and 1).  A geometric sub-bin mean is the exponential
    of the mean of its elementary log means; an arithmetic one the mean of
    its elementary means (every elementary sub-bin has the same width)."""
    import numpy as np
    idx = [0] + [int(round(b * n_elem)) for b in borders] + [n_elem]
    x = np.log(elem) if mean == "geometric" else np.asarray(elem, dtype=np.float64)
    c = np.concatenate([np.zeros(x.shape[:-1] + (1,)), np.cumsum(x, axis=-1)], axis=-1)
    out = np.stack([(c[..., b] - c[..., a]) / (b - a) for a, b in zip(idx[:-1], idx[1:])], axis=-1)
    return np.exp(out) if mean == "geometric" else out


def slab_columns(kappa_c, tau_c=SLAB_TAU_C):
    """Column masses m [B][C] (g cm^-2) with continuum optical depths tau_c."""
    import numpy as np
    return np.asarray(tau_c, dtype=np.float64)[None, :] / np.asarray(kappa_c, dtype=np.float64)[:, None]


def slab_odf_errors(steps, fracs, fine_I, kappa_c, columns):
    """|I_ODF / I_N - 1| [P][B][C] for ODF steps [P][B][S] with width
    fractions fracs; fine_I [P][B][C] holds the fine-grid bin intensities
    I_N, kappa_c [B] the continuum at bin centres, columns [B][C] the column
    masses.  I(kappa) = 1 - exp(-(kappa + kappa_c) m) (isothermal slab, in
    units of the Planck function)."""
    import numpy as np
    f = np.asarray(fracs, dtype=np.float64)
    k = steps[..., None, :] + kappa_c[None, :, None, None]          # [P][B][1][S]
    I = np.sum(f * -np.expm1(-k * columns[None, :, :, None]), axis=-1)   # [P][B][C]
    return np.abs(I / fine_I - 1.0)


def slab_odf_error(steps, fracs, fine_I, kappa_c, columns):
    """max |I_ODF / I_N - 1| over points, bins and columns."""
    return float(slab_odf_errors(steps, fracs, fine_I, kappa_c, columns).max())


def _error_stats(e):
    import numpy as np
    return dict(max=float(e.max()), p95=float(np.percentile(e, 95.0)), median=float(np.median(e)))


def run_subbins(args):
    """Flexible few-step ODFs (Sec. 4.1): the best borders of 2-4 sub-bins,
    found by search on training points, against the standard 12 sub-bins,
    judged by an isothermal slab (Sec. 2.3 I_ODF against the fine-grid I_N)."""
    import itertools
    import numpy as np
    import torch
    from dataclasses import replace
    from paper_2105_13611_amd import odf
    from paper_2105_13611_amd import workload as W
    lo, hi = args.pretab_nm
    n_lines = int(round(1e7 * math.log(hi / lo) / math.log(W.LAMBDA_LAST_FULL_NM / 9.0)))
    N = W.grid_size(lo, hi, W.RESOLVING_POWER)
    nb = max(1, N // 2000)
    base = W.config(2, n_lines=n_lines, lam_range=(lo, hi), n_bins=nb)
    edges = base.layout.bin_edges
    g = W.dfsynthe_tp_grid()
    sel = np.nonzero((g.T_K >= 3000.0) & (g.T_K <= 20000.0) & (g.log10_P >= 0.0) & (g.log10_P <= 7.0))[0]
    rng = np.random.default_rng(5)
    pick = np.sort(rng.choice(sel, size=min(args.subbin_points, sel.size), replace=False))
    pts = g.take(pick)
    train = np.arange(pts.n_points) % 2 == 0
    ws = int(min(args.workspace_gb, 8.0) * (1 << 30))
    prec = "mixed" if args.precision == "both" else args.precision
    t0 = time.perf_counter()
    # the floored fine-grid opacity and the fine-grid slab intensity per bin
    with odf.plan_for(replace(base, options=replace(base.options, output="fine")), precision=prec,
                      workspace_bytes=ws) as pf:
        fine, _ = pf.compute(base.species.abundance, pts)
    lam_c = base.layout.lambda_first_nm * np.exp(0.5 * (edges[:-1] + edges[1:] - 1) * math.log1p(1.0 / W.RESOLVING_POWER))
    o = base.options
    kc = o.kappa_c_ref * (lam_c / o.lambda_c_ref_nm) ** o.kappa_c_power
    kc_t = torch.as_tensor(kc, device=fine.device)
    bin_of = torch.as_tensor(np.repeat(np.arange(nb), np.diff(edges)), device=fine.device)
    widths = torch.as_tensor(np.diff(edges).astype(np.float64), device=fine.device)
    kf = fine[:, int(edges[0]):int(edges[-1])].double()
    cols = slab_columns(kc)
    fine_I = np.empty((pts.n_points, nb, len(SLAB_TAU_C)))
    for c in range(len(SLAB_TAU_C)):
        m = torch.as_tensor(cols[:, c], device=fine.device)[bin_of]
        I = -torch.expm1(-(kf + kc_t[bin_of]) * m)
        acc = torch.zeros(pts.n_points, nb, dtype=torch.float64, device=fine.device)
        acc.index_add_(1, bin_of, I)
        fine_I[:, :, c] = (acc / widths).cpu().numpy()
    del fine, kf
    # ODFs: the standard 12 sub-bins, and elementary sub-bins for the search
    res = {}
    elem = {}
    for mean in ("geometric", "arithmetic"):
        lay12 = replace(base.layout, step_frac=W.STEP_FRAC_12.copy())
        with odf.plan_for(replace(base, layout=lay12, options=replace(base.options, mean=mean)),
                          precision=prec, workspace_bytes=ws) as p12:
            s12, _ = p12.compute(base.species.abundance, pts)
        s12 = s12.double().cpu().numpy()
        laye = replace(base.layout, step_frac=np.full(N_ELEMENTARY, 1.0 / N_ELEMENTARY))
        with odf.plan_for(replace(base, layout=laye, options=replace(base.options, mean=mean)),
                          precision=prec, workspace_bytes=ws) as pe:
            se, _ = pe.compute(base.species.abundance, pts)
        elem[mean] = se.double().cpu().numpy()
        std_b = np.cumsum(W.STEP_FRAC_12)[:-1]
        s12e = combine_steps(elem[mean], std_b, mean)
        res[f"12_standard_{mean}"] = dict(
            borders=[round(float(b), 4) for b in std_b],
            train=_error_stats(slab_odf_errors(s12[train], W.STEP_FRAC_12, fine_I[train], kc, cols)),
            test=_error_stats(slab_odf_errors(s12[~train], W.STEP_FRAC_12, fine_I[~train], kc, cols)),
            from_elementary_max_rel_diff=float(np.max(np.abs(s12e / s12 - 1.0))))
        # search: the borders with the least 95th-percentile error on the
        # training points (the paper's claim is for most of the range)
        for n_s in (2, 3, 4):
            best = None
            for bs in itertools.combinations(BORDER_CANDIDATES, n_s - 1):
                fr = np.diff(np.concatenate([[0.0], bs, [1.0]]))
                e = slab_odf_errors(combine_steps(elem[mean][train], bs, mean), fr, fine_I[train], kc, cols)
                obj = float(np.percentile(e, 95.0))
                if best is None or obj < best[0]:
                    best = (obj, bs, fr, e)
            e_test = slab_odf_errors(combine_steps(elem[mean][~train], best[1], mean), best[2],
                                     fine_I[~train], kc, cols)
            res[f"{n_s}_best_{mean}"] = dict(borders=list(best[1]), train=_error_stats(best[3]),
                                             test=_error_stats(e_test))
        log(f"[bench] sub-bins ({mean}), test max / p95 / median: " + ", ".join(
            f"{k}: {v['test']['max']:.2e} / {v['test']['p95']:.2e} / {v['test']['median']:.2e}"
            for k, v in res.items() if k.endswith(mean)))
    dt = time.perf_counter() - t0
    return {
        "metric": SUBBIN_METRIC, "value": res["3_best_geometric"]["test"]["max"], "unit": "relative",
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": dt * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": f"{lo}-{hi} nm at R=5e5 ({N} fine points) in {nb} bins of about 2000 points, "
                               f"{n_lines} synthetic lines, {pts.n_points} T-P points of the 57 x 25 table "
                               f"(3000-20000 K, log P 0-7; even ones train the borders, odd ones test them)",
                   "points": pts.n_points, "bins": nb, "continuum_tau": list(SLAB_TAU_C)},
        "value_is": "max error on the test points of the best 3-sub-bin geometric ODF",
        "configurations": res,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["table", "serve", "pretab", "subbins"], default="table")
    ap.add_argument("--subbin-points", type=int, default=40, help="T-P points of --mode subbins")
    ap.add_argument("--pretab-nm", type=float, nargs=2, default=[300.0, 450.0],
                    help="wavelength interval of --mode pretab (nm)")
    ap.add_argument("--no-interp", action="store_true", help="--mode pretab without the interpolation study")
    ap.add_argument("--serve-requests", type=int, default=12)
    ap.add_argument("--serve-rate", type=float, default=0.0, help="req/s (0 = the stream's 20 req/s)")
    ap.add_argument("--serve-max-points", type=int, default=0)
    ap.add_argument("--serve-config", type=int, choices=[4, 5], default=4,
                    help="4: Poisson stream over 1e7 lines; 5: bursts over 1e8 lines")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["both", "mixed", "fp64"], default="both")
    ap.add_argument("--fp64-steps", type=int, default=2,
                    help="timed steps of the plain FP64 leg (about 25 s each on the full table)")
    ap.add_argument("--fp64-warmup", type=int, default=1, help="untimed steps of the plain FP64 leg")
    ap.add_argument("--points", type=int, default=0, help="stratified subset (0 = whole table)")
    ap.add_argument("--workspace-gb", type=float, default=80.0)
    ap.add_argument("--batch-points", type=int, default=0, help="points per device batch (0 = automatic)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-kernel-alone", action="store_true",
                    help="skip the Voigt-alone timing (profiled runs: counters then cover the table only)")
    ap.add_argument("--cpu-workers", type=int, default=0)
    ap.add_argument("--config", type=int, choices=sorted(WORKLOADS), default=2,
                    help="2: the 1425-point table (default); 3: the same at five vturb (7125 points); "
                         "5: 1e8 lines over 80 species x 3 stages (use --points and a larger --workspace-gb)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="first copy a buffer of this size three times (a reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the ODF table shards over points with no exchange; see the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.mode == "table":
        run_table(args)
        return
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    copy_calibration(args)
    if args.mode == "pretab":
        print(json.dumps(run_pretab(args)), flush=True)
        return
    if args.mode == "subbins":
        print(json.dumps(run_subbins(args)), flush=True)
        return
    print(json.dumps(run_serving(args.serve_requests, args.serve_rate, args.workspace_gb,
                                 args.serve_max_points, args.serve_config)), flush=True)


def copy_calibration(args):
    """Optionally copy a buffer of known size three times (the reference
    for rocprofv3's HBM byte counters)."""
    import torch
    if not args.copy_calibration_mb:
        return
    n = args.copy_calibration_mb << 18   # float32 elements
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)   # an elementwise kernel (a same-type copy_ may use DMA)
    torch.cuda.synchronize()
    log(f"[bench] copy calibration: 3 copies of {args.copy_calibration_mb} MiB")
    del a, b


def run_table(args):
    """The table benchmark: the CPU leg first (before anything touches the
    GPU), then the mixed leg at the given steps, then the plain FP64 leg at
    its bounded steps; one JSON line."""
    from paper_2105_13611_amd import workload as W
    t0 = time.perf_counter()
    w = W.config(args.config)
    log(f"[bench] workload generated in {time.perf_counter() - t0:.1f} s: {w.lines.n_lines} lines, "
        f"{w.points.n_points} points, {w.layout.n_bins} bins")
    idx = None if args.points == 0 else stratified_points(w.points, args.points)
    cpu, ref, sbins = None, None, None
    if not args.no_cpu:
        workers = args.cpu_workers or min(16, os.cpu_count() or 1)
        log(f"[bench] CPU baseline: oracle on {workers} processes")
        cpu, ref, sbins = cpu_baseline(w, workers)
        log(f"[bench] CPU baseline: {cpu['value']:.4f} points/s, wall {cpu['wall_s']:.1f} s")
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    copy_calibration(args)
    sample = None if ref is None else (sorted(ref), sbins)
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    res = {}
    for p in precs:
        steps, warmup = ((args.steps, args.warmup) if p == precs[0] or p == "mixed"
                         else (args.fp64_steps, args.fp64_warmup))
        res[p] = run_gpu(w, p, steps, warmup, args.workspace_gb, idx, args.batch_points, sample,
                         alone=not args.no_kernel_alone)
        r = res[p]
        log(f"[bench] {p}: {r['n_points'] * r['steps'] / r['seconds']:.2f} points/s, "
            f"stage ms {r['stage_ms']}, plan {r['plan_seconds']:.1f} s")
    head = res[precs[0]]
    n_pts = head["n_points"]
    value = n_pts * head["steps"] / head["seconds"]
    line_evals = head["stats"]["line_evals"] * head["steps"] / head["seconds"]
    rl = roofline(head, FLOP_PER_SAMPLE_F32 if precs[0] == "mixed" else FLOP_PER_SAMPLE_F64, precs[0])
    out = {
        "metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": head["steps"],
        "warmup": head["warmup"], "ms_per_step": head["seconds"] / head["steps"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if precs[0] == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config]
                   + ("" if idx is None else f" [stratified subset of {n_pts} points]"),
                   "points": n_pts, "lines": w.lines.n_lines, "grid_points": int(w.layout.bin_edges[-1]),
                   "bins": w.layout.n_bins, "sub_bins": w.layout.n_steps},
        "line_evals_per_s": line_evals,
        "voigt_samples_per_s": head["stats"]["voigt_samples"] * head["steps"] / head["seconds"],
        "survivors_per_point": head["stats"]["survivors"] / n_pts,
        "voigt_samples_per_point": head["stats"]["voigt_samples"] / n_pts,
        "roofline": rl,
    }
    for p in precs:
        r = res[p]
        out[f"{p}_path"] = dict(points_per_s=r["n_points"] * r["steps"] / r["seconds"],
                                line_evals_per_s=r["stats"]["line_evals"] * r["steps"] / r["seconds"],
                                seconds_per_step=r["seconds"] / r["steps"], steps=r["steps"],
                                warmup=r["warmup"],
                                stage_ms={k: v["ms"] for k, v in r["stage_ms"].items()},
                                stage_busy_ms={k: v["busy_ms"] for k, v in r["stage_ms"].items()},
                                plan_seconds=r["plan_seconds"], checksum=r["checksum"])
    if "fp64" in res and "mixed" in res:
        out["mixed_over_fp64_speedup"] = out["mixed_path"]["points_per_s"] / out["fp64_path"]["points_per_s"]
        out["roofline_fp64"] = roofline(res["fp64"], FLOP_PER_SAMPLE_F64, "fp64")
    if ref is not None:
        out["parity"] = parity_block(ref, sbins, {p: res[p].get("sample_out", {}) for p in precs})
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

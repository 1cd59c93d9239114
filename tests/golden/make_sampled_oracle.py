"""Write the oracle's ODF steps at sampled (point, bin) pairs of the two large
workloads to JSON fixtures beside this script.

Calls only the oracle and the seeded workload generator (which holds no
physics); nothing here touches the HIP path.  The GPU tests regenerate the
same seeded inputs, run them through the library and compare with these
values, so the slow FP64 oracle does not have to run on the GPU host.

  cfg4_served_oracle.json   the first four requests of the serving stream
                            (1e7 lines, 40 species x 2 stages, each request
                            with its own [M/H], [alpha/Fe] and 762-1025 T-P
                            points): 8 points of each, evenly spaced over its
                            point list, x 64 bins evenly spaced over the 1212
  cfg5_sampled_oracle.json  the first four requests of the 1e8-line stream
                            (80 species x 3 stages, each with its own
                            composition over the 57 x 25 x 5 grid): 8 points
                            of each, drawn with a seeded generator, x the
                            same 64 bins

For each pair the oracle's 12 steps and whether the bin holds a near-tie
decision (a keep test or window edge within rounding of its boundary; there
the test recomputes the reference with the GPU's own decisions).

The oracle only needs the lines that can reach a sampled bin at that point
(tests/gpu_helpers.Reach: a window spans at most 500 Doppler widths of the
lightest species at the point's T and v_turb).

Usage: python tests/golden/make_sampled_oracle.py [cfg4] [cfg5] [--workers N]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2105_13611_amd import workload as W  # noqa: E402
from tests.gpu_helpers import Reach, ambiguous_bins  # noqa: E402

BINS = 64           # bins per point, evenly spaced over the layout's
POINTS = 8          # points per request
REQUESTS = 4

_G = {}


def _task(args):
    """One point: each bin with the lines that can reach it (memory stays at
    one bin's reach even for the 1e8-line list)."""
    abundance, T, lp, v = args
    g = _G
    steps, tie, n_reach = [], [], 0
    for b in g["bins"]:
        sub = g["reach"].lines_for([b], T, v)
        st, _, ex = oracle.odf_point(g["lines"].take(sub), g["species"], abundance, T, lp, v, g["layout"],
                                     g["options"], [b])
        steps.append(st[0])
        tie.append(int(b) in ambiguous_bins(ex["lq"], g["layout"].bin_edges))
        n_reach += int(sub.size)
    return steps, tie, n_reach


def _run(w, bins, tasks, workers):
    """Oracle steps of every task, in task order; the hottest points start
    first so the pool's tail is short."""
    _G.update(lines=w.lines, species=w.species, layout=w.layout, options=w.options, bins=list(bins),
              reach=Reach(w.lines, w.species, w.layout, w.options))
    order = sorted(range(len(tasks)), key=lambda k: -tasks[k][1])
    with mp.get_context("fork").Pool(workers) as pool:
        out = pool.map(_task, [tasks[k] for k in order], chunksize=1)
    _G.clear()
    res = [None] * len(tasks)
    for k, r in zip(order, out):
        res[k] = r
    return res


def _bins(w):
    return [int(b) for b in np.round(np.linspace(0, w.layout.n_bins - 1, BINS))]


def _f(a):
    return [float(x) for x in np.asarray(a).ravel()]


def _requests(w, pick):
    """Per request: its sampled points (pick(rid, request) -> indices into its
    point list) and the oracle tasks for them."""
    reqs, tasks = [], []
    for rid, r in enumerate(w.requests):
        idx = pick(rid, r)
        pts = r.points.take(idx)
        reqs.append(dict(id=rid, n_points=r.points.n_points, point_index=[int(i) for i in idx],
                         T_K=_f(pts.T_K), log10_P=_f(pts.log10_P), vturb_kms=_f(pts.vturb_kms),
                         abundance=_f(r.abundance)))
        tasks += [(r.abundance, float(pts.T_K[k]), float(pts.log10_P[k]), float(pts.vturb_kms[k]))
                  for k in range(pts.n_points)]
    return reqs, tasks


def _fill(reqs, res):
    k = 0
    for q in reqs:
        n = len(q["point_index"])
        q["steps"] = [[_f(s) for s in res[k + j][0]] for j in range(n)]
        q["near_tie"] = [res[k + j][1] for j in range(n)]
        q["line_bin_pairs_in_reach"] = [res[k + j][2] for j in range(n)]
        k += n


SOURCE = ("FP64 oracle (oracle/) ODF steps, written by tests/golden/make_sampled_oracle.py from the seeded "
          "workload generator; no value comes from the HIP path")


def cfg4(workers):
    w = W.config(4, n_requests=REQUESTS)
    bins = _bins(w)
    reqs, tasks = _requests(w, lambda rid, r: np.unique(
        np.round(np.linspace(0, r.points.n_points - 1, POINTS)).astype(np.int64)))
    t0 = time.perf_counter()
    _fill(reqs, _run(w, bins, tasks, workers))
    return dict(_source=SOURCE,
                workload=(f"serving stream over the 1e7-line list: requests 0-{REQUESTS - 1} (seeded), "
                          f"{POINTS} points each evenly spaced over the request's list, {BINS} bins evenly "
                          "spaced over the 1212"),
                config=4, bins=bins, oracle_seconds=time.perf_counter() - t0, requests=reqs)


def cfg5(workers):
    w = W.config(5, n_requests=REQUESTS)
    bins = _bins(w)
    reqs, tasks = _requests(w, lambda rid, r: np.sort(
        np.random.default_rng(5_000 + rid).choice(r.points.n_points, POINTS, replace=False)))
    t0 = time.perf_counter()
    _fill(reqs, _run(w, bins, tasks, workers))
    return dict(_source=SOURCE,
                workload=(f"1e8-line stream (80 species x 3 stages): requests 0-{REQUESTS - 1} (seeded "
                          f"compositions), {POINTS} points each of the 57 x 25 x 5 grid drawn with "
                          f"default_rng(5000 + request), {BINS} bins evenly spaced over the 1212"),
                config=5, bins=bins, oracle_seconds=time.perf_counter() - t0, requests=reqs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["cfg4", "cfg5"])
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    for name in args.which:
        d = {"cfg4": cfg4, "cfg5": cfg5}[name](args.workers)
        path = os.path.join(HERE, f"{name}_{'served' if name == 'cfg4' else 'sampled'}_oracle.json")
        with open(path, "w") as fh:
            json.dump(d, fh, separators=(",", ":"))
        print(f"{path}: oracle {d['oracle_seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    main()

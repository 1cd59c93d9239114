"""Write the oracle's ODF steps at sampled (point, bin) pairs of the two large
workloads to JSON fixtures beside this script.

Calls only the oracle and the seeded workload generator (which holds no
physics); nothing here touches the HIP path.  The GPU tests regenerate the
same seeded inputs, run them through the library and compare with these
values, so the slow FP64 oracle does not have to run on the GPU host.

  cfg4_served_oracle.json   the first four requests of the serving stream
                            (1e7 lines, 40 species x 2 stages, each request
                            with its own [M/H], [alpha/Fe] and 762-1025 T-P
                            points): 4 points of each, evenly spaced over its
                            point list, x 16 bins evenly spaced over the 1212
  cfg5_sampled_oracle.json  the 1e8-line list (80 species x 3 stages) with the
                            first request's composition: 4 T-P-v_turb points
                            of the grid x 8 bins evenly spaced

For each pair the oracle's 12 steps and whether the bin holds a near-tie
decision (a keep test or window edge within rounding of its boundary; there
the test recomputes the reference with the GPU's own decisions).

The oracle only needs the lines that can reach a sampled bin: a window spans
at most 500 Doppler widths, under 3.2 % in wavelength on these grids (2e5 K,
12 amu, 8 km/s), so the lines within 5 % of a bin's wavelengths are a
superset of them.

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
from tests.gpu_helpers import ambiguous_bins  # noqa: E402

REACH = 1.05

_G = {}


def reach_subset(lines, layout, bins):
    """Indices of the lines within REACH of any of the bins' wavelengths."""
    e = layout.bin_edges
    lam = lines.lambda_nm
    keep = np.zeros(lam.size, dtype=bool)
    for b in bins:
        l0 = float(oracle.grid_lambda_nm(layout, e[b]))
        l1 = float(oracle.grid_lambda_nm(layout, e[b + 1] - 1))
        keep |= (lam > l0 / REACH) & (lam < l1 * REACH)
    return np.nonzero(keep)[0]


def _task(args):
    abundance, T, lp, v = args
    g = _G
    steps, _, ex = oracle.odf_point(g["lines"], g["species"], abundance, T, lp, v, g["layout"],
                                    g["options"], g["bins"])
    amb = ambiguous_bins(ex["lq"], g["layout"].bin_edges)
    return steps, [int(b) in amb for b in g["bins"]]


def _run(w, sub, bins, tasks, workers):
    _G.update(lines=w.lines.take(sub), species=w.species, layout=w.layout,
              options=w.options, bins=list(bins))
    with mp.get_context("fork").Pool(workers) as pool:
        res = pool.map(_task, tasks, chunksize=1)
    _G.clear()
    return res


def _f(a):
    return [float(x) for x in np.asarray(a).ravel()]


def cfg4(workers):
    w = W.config(4, n_requests=4)
    bins = [int(b) for b in np.round(np.linspace(0, w.layout.n_bins - 1, 16))]
    sub = reach_subset(w.lines, w.layout, bins)
    reqs, tasks = [], []
    for rid, r in enumerate(w.requests):
        idx = np.unique(np.round(np.linspace(0, r.points.n_points - 1, 4)).astype(np.int64))
        pts = r.points.take(idx)
        reqs.append(dict(id=rid, n_points=r.points.n_points, point_index=[int(i) for i in idx],
                         T_K=_f(pts.T_K), log10_P=_f(pts.log10_P), vturb_kms=_f(pts.vturb_kms),
                         abundance=_f(r.abundance)))
        tasks += [(r.abundance, float(pts.T_K[k]), float(pts.log10_P[k]), float(pts.vturb_kms[k]))
                  for k in range(pts.n_points)]
    t0 = time.perf_counter()
    res = _run(w, sub, bins, tasks, workers)
    k = 0
    for q in reqs:
        n = len(q["point_index"])
        q["steps"] = [[_f(s) for s in res[k + j][0]] for j in range(n)]
        q["near_tie"] = [res[k + j][1] for j in range(n)]
        k += n
    return dict(_source=("FP64 oracle (oracle/) ODF steps, written by tests/golden/make_sampled_oracle.py "
                         "from the seeded workload generator; no value comes from the HIP path"),
                workload=("serving stream over the 1e7-line list: requests 0-3 (seeded), 4 points each "
                          "evenly spaced over the request's list, 16 bins evenly spaced over the 1212"),
                config=4, bins=bins, lines_in_reach=int(sub.size), oracle_seconds=time.perf_counter() - t0,
                requests=reqs)


# T-P-v points of the 57 x 25 x 5 grid: (T index, log P index, v_turb)
CFG5_POINTS = [(4, 24, 0.0), (18, 10, 1.0), (36, 16, 4.0), (56, 2, 8.0)]


def cfg5(workers):
    w = W.config(5, n_requests=1)
    T = 2000.0 * 100.0 ** (np.array([p[0] for p in CFG5_POINTS]) / 56.0)
    lp = -4.0 + 0.5 * np.array([p[1] for p in CFG5_POINTS], dtype=np.float64)
    v = np.array([p[2] for p in CFG5_POINTS])
    bins = [int(b) for b in np.round(np.linspace(0, w.layout.n_bins - 1, 8))]
    sub = reach_subset(w.lines, w.layout, bins)
    a = w.requests[0].abundance
    tasks = [(a, float(T[i]), float(lp[i]), float(v[i])) for i in range(T.size)]
    t0 = time.perf_counter()
    res = _run(w, sub, bins, tasks, min(workers, len(tasks)))
    return dict(_source=("FP64 oracle (oracle/) ODF steps, written by tests/golden/make_sampled_oracle.py "
                         "from the seeded workload generator; no value comes from the HIP path"),
                workload=("1e8-line list (80 species x 3 stages) with request 0's composition: 4 points "
                          "of the 57 x 25 x 5 grid x 8 bins evenly spaced over the 1212"),
                config=5, request=0, bins=bins, lines_in_reach=int(sub.size),
                oracle_seconds=time.perf_counter() - t0,
                T_K=_f(T), log10_P=_f(lp), vturb_kms=_f(v), abundance=_f(a),
                steps=[[_f(s) for s in r[0]] for r in res], near_tie=[r[1] for r in res])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="*", default=["cfg4", "cfg5"])
    ap.add_argument("--workers", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    for name in args.which:
        d = {"cfg4": cfg4, "cfg5": cfg5}[name](args.workers)
        path = os.path.join(HERE, f"{name}_{'served' if name == 'cfg4' else 'sampled'}_oracle.json")
        with open(path, "w") as fh:
            json.dump(d, fh, indent=1)
        print(f"{path}: {d['lines_in_reach']} lines in reach, oracle {d['oracle_seconds']:.0f} s", flush=True)


if __name__ == "__main__":
    main()

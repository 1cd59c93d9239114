"""Shared helpers of the GPU tests: oracle-side ambiguity detection.

Where floating point decides an integer (a line kept or not, a window edge
rounded up or down) the HIP path and the oracle may take different, equally
valid decisions when the real value sits within rounding of the boundary.
These helpers find such cases from the oracle's real-valued decisions so the
tests compare what is unique and check that the rest is valid.
"""
import math

import numpy as np

import oracle

KEEP_RTOL = 1e-11      # |core/thr - 1| below this: either keep decision is valid
EDGE_ATOL = 1e-7       # real window edge this close to an integer: +-1 is valid


def ambiguous_lines(lq):
    """Boolean mask over lines whose decisions are within rounding of a boundary."""
    with np.errstate(divide="ignore", invalid="ignore"):
        keep_tie = np.abs(lq["core"] / lq["thr"] - 1.0) < KEEP_RTOL
    lo_tie = np.abs(lq["jlo_r"] - np.round(lq["jlo_r"])) < EDGE_ATOL
    hi_tie = np.abs(lq["jhi_r"] - np.round(lq["jhi_r"])) < EDGE_ATOL
    return keep_tie, lo_tie & lq["keep"], hi_tie & lq["keep"]


def ambiguous_points(lq, N):
    """Fine-grid indices whose line opacity depends on an ambiguous decision."""
    keep_tie, lo_tie, hi_tie = ambiguous_lines(lq)
    pts = set()
    for i in np.nonzero(keep_tie & (lq["jlo"] <= lq["jhi"]))[0]:
        pts.update(range(int(lq["jlo"][i]), int(lq["jhi"][i]) + 1))
    for i in np.nonzero(lo_tie)[0]:
        j = int(round(lq["jlo_r"][i]))
        pts.update(k for k in (j - 1, j, j + 1) if 0 <= k < N)
    for i in np.nonzero(hi_tie)[0]:
        j = int(round(lq["jhi_r"][i]))
        pts.update(k for k in (j - 1, j, j + 1) if 0 <= k < N)
    return np.array(sorted(pts), dtype=np.int64)


def ambiguous_bins(lq, edges):
    pts = ambiguous_points(lq, int(edges[-1]))
    if pts.size == 0:
        return set()
    b = np.searchsorted(edges, pts, side="right") - 1
    return set(int(x) for x in b if 0 <= x < len(edges) - 1)


def floor_values(layout, opts, j0, j1):
    return opts.cutoff * oracle.physics.kappa_c(oracle.grid_lambda_nm(layout, np.arange(j0, j1)), opts)


def rel_err(got, ref):
    return np.abs(np.asarray(got, dtype=np.float64) / np.asarray(ref, dtype=np.float64) - 1.0)


def log10_err(got, ref):
    return np.abs(np.log10(np.asarray(got, dtype=np.float64)) - np.log10(np.asarray(ref, dtype=np.float64)))


def fmt(x):
    return f"{x:.3e}" if isinstance(x, float) and math.isfinite(x) else str(x)


def compare_points(w, out, prec, bins=None, abundance=None):
    """Largest relative and log10 errors of out[point][bin][step] against the
    oracle's ODF, and the number of bins skipped as ambiguous."""
    a = w.species.abundance if abundance is None else abundance
    worst, worst_log, skipped = 0.0, 0.0, 0
    for i in range(w.points.n_points):
        ref, _, ex = oracle.odf_point(w.lines, w.species, a, float(w.points.T_K[i]),
                                      float(w.points.log10_P[i]), float(w.points.vturb_kms[i]),
                                      w.layout, w.options, bins)
        bsel = np.arange(w.layout.n_bins) if bins is None else np.asarray(bins)
        amb = ambiguous_bins(ex["lq"], w.layout.bin_edges)
        got = out[i][bsel]
        for k, b in enumerate(bsel):
            if int(b) in amb:
                skipped += 1
                continue
            worst = max(worst, float(rel_err(got[k], ref[k]).max()))
            worst_log = max(worst_log, float(log10_err(got[k], ref[k]).max()))
    return worst, worst_log, skipped

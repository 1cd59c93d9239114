"""High-resolution line opacity and the ODF reduction.  TEST INFRASTRUCTURE ONLY.

* Grid: lambda_j = lambda_first q^j, q = 1 + 1/R, j = 0..N-1 (App. E grid
  formula, written 0-based).
* Line opacity on the grid: every kept line adds S * H(x_j, a) inside its
  window, x_j = (nu_j - nu_0)/dnu_D taken exactly from the index as
  expm1((j* - j) ln q)/b (Sec. 2.1, eq. l_nu_line; App. E second stage).
* Floor at the selection level cutoff * kappa_c(lambda_j): values below it
  are unresolved by construction of the pre-selection (Sec. 4.3).
* ODF: within each bin the opacities are sorted ascending and split into
  sub-bins whose widths are given fractions of the bin; each sub-bin is
  averaged with the geometric mean (the paper's default) or the arithmetic
  mean (Sec. 2.3; App. E third stage; App. G keyword 'mean arithmetic').  A
  sorted point i covers [i, i+1) on the sorted axis and contributes to a
  sub-bin with the length of the overlap, so fractional sub-bin borders are
  honoured exactly.
* Pre-tabulated high-resolution opacity (Sec. 4.1, option to pre-tabulate):
  the table in ODF form with one sub-bin per fine point, i.e. the floored
  opacity of every point of the grid.
* A consumer of the ODF with no dataset: the emergent intensity of an
  isothermal slab of column mass m, in units of the Planck function,
  I(kappa) = 1 - exp(-(kappa + kappa_c) m).  The bin intensity from the fine
  grid is the equal-weight mean over the bin's points (the sum I_N of
  Sec. 2.3 with the bin's steps taken as equal); from the ODF it is the sum
  over sub-bins weighted by their widths (Sec. 2.3, I_ODF; App. E, the
  weighted sum over sub-bins with the continuum added to every sub-bin).
"""
import math

import numpy as np

from .physics import grid_size, kappa_c, line_quantities
from .voigt import voigt_h

__all__ = ["grid_size", "grid_lambda_nm", "fine_opacity", "odf_reduce_bin",
           "odf_point", "odf", "fine_table_point", "slab_fine_intensity", "slab_odf_intensity"]

_CHUNK_SAMPLES = 4_000_000


def grid_lambda_nm(layout, j):
    lnq = math.log1p(1.0 / layout.resolving_power)
    return layout.lambda_first_nm * np.exp(np.asarray(j, dtype=np.float64) * lnq)


def fine_opacity(lq, layout, j0, j1):
    """Line opacity kappa_l[j] for j in [j0, j1) from the kept lines in lq.

    A plain scatter-sum: for every line whose window meets [j0, j1), every
    sample of the overlap adds S * H(x_j, a).
    """
    out = np.zeros(j1 - j0, dtype=np.float64)
    lnq = math.log1p(1.0 / layout.resolving_power)
    sel = lq["surv"] & (lq["jlo"] <= j1 - 1) & (lq["jhi"] >= j0)
    idx = np.nonzero(sel)[0]
    if idx.size == 0:
        return out
    lo = np.maximum(lq["jlo"][idx], j0)
    hi = np.minimum(lq["jhi"][idx], j1 - 1)
    cnt = hi - lo + 1
    # chunk the lines so that no chunk holds more than _CHUNK_SAMPLES samples
    csum = np.cumsum(cnt)
    start = 0
    while start < idx.size:
        base = csum[start - 1] if start > 0 else 0
        stop = int(np.searchsorted(csum, base + _CHUNK_SAMPLES, side="right"))
        stop = max(stop, start + 1)
        ii = idx[start:stop]
        c = cnt[start:stop]
        rep = np.repeat(np.arange(ii.size), c)
        first = np.repeat(np.cumsum(c) - c, c)
        j = np.repeat(lo[start:stop], c) + (np.arange(rep.size) - first)
        line = ii[rep]
        x = np.expm1((lq["jstar"][line] - j) * lnq) / lq["b"][line]
        val = lq["S"][line] * voigt_h(x, lq["a"][line])
        out += np.bincount(j - j0, weights=val, minlength=j1 - j0)
        start = stop
    return out


def odf_reduce_bin(values, step_frac, mean="geometric"):
    """ODF steps of one bin: sort ascending, overlap-weighted sub-bin means.

    Sub-bin s spans [F_{s-1} n, F_s n) on the sorted axis, F the cumulative
    fractions (normalised to end at exactly 1); sorted point i spans [i, i+1).
    """
    v = np.sort(np.asarray(values, dtype=np.float64))
    n = v.size
    F = np.concatenate([[0.0], np.cumsum(step_frac)])
    F = F / F[-1]
    B = F * n
    i = np.arange(n, dtype=np.float64)
    g = np.log(v) if mean == "geometric" else v
    out = np.empty(len(step_frac))
    for s in range(len(step_frac)):
        w = np.clip(np.minimum(i + 1.0, B[s + 1]) - np.maximum(i, B[s]), 0.0, None)
        m = np.sum(w * g) / (B[s + 1] - B[s])
        out[s] = math.exp(m) if mean == "geometric" else m
    return out


def odf_point(lines, species, abundance, T, log10_P, vturb, layout, opts,
              bins=None, return_fine=False):
    """ODF steps for one (T, P, v) point over the bins listed (all if None).

    Returns (steps[n_bins_sel, n_steps], counters, extra) where counters holds
    line_evals, survivors and voigt_samples over the whole grid.
    """
    lq = line_quantities(lines, species, abundance, T, log10_P, vturb, layout, opts)
    edges = np.asarray(layout.bin_edges, dtype=np.int64)
    nb = edges.size - 1
    bins = np.arange(nb) if bins is None else np.asarray(bins, dtype=np.int64)
    steps = np.empty((bins.size, len(layout.step_frac)))
    fine = {}
    for k, bidx in enumerate(bins):
        j0, j1 = int(edges[bidx]), int(edges[bidx + 1])
        kl = fine_opacity(lq, layout, j0, j1)
        floor = opts.cutoff * kappa_c(grid_lambda_nm(layout, np.arange(j0, j1)), opts)
        kt = np.maximum(kl, floor)
        steps[k] = odf_reduce_bin(kt, layout.step_frac, opts.mean)
        if return_fine:
            fine[int(bidx)] = (kl, kt)
    s = lq["surv"]
    counters = dict(line_evals=int(lines.n_lines), survivors=int(np.count_nonzero(s)),
                    voigt_samples=int(np.sum(lq["jhi"][s] - lq["jlo"][s] + 1)))
    extra = dict(lq=lq, fine=fine)
    return steps, counters, extra


def fine_table_point(lines, species, abundance, T, log10_P, vturb, layout, opts, j0=0, j1=None):
    """Pre-tabulated opacity of one point on fine points [j0, j1): each fine
    point is a bin of its own with a single sub-bin, whose mean is the
    floored opacity max(kappa_l, cutoff kappa_c) of that point."""
    lq = line_quantities(lines, species, abundance, T, log10_P, vturb, layout, opts)
    j1 = lq["N"] if j1 is None else j1
    kl = fine_opacity(lq, layout, j0, j1)
    floor = opts.cutoff * kappa_c(grid_lambda_nm(layout, np.arange(j0, j1)), opts)
    return np.maximum(kl, floor), lq


def slab_fine_intensity(kappa_bin, kappa_c, column):
    """Fine-grid bin intensity of the slab: mean over the bin of
    1 - exp(-(kappa_j + kappa_c) m), for every column m given."""
    k = np.asarray(kappa_bin, dtype=np.float64)[None, :]
    m = np.atleast_1d(np.asarray(column, dtype=np.float64))[:, None]
    return np.mean(-np.expm1(-(k + kappa_c) * m), axis=1)


def slab_odf_intensity(steps, step_frac, kappa_c, column):
    """ODF bin intensity of the slab: sum over sub-bins of their width
    fraction times 1 - exp(-(kappa_s + kappa_c) m)."""
    f = np.asarray(step_frac, dtype=np.float64)
    f = f / f.sum()
    k = np.asarray(steps, dtype=np.float64)[None, :]
    m = np.atleast_1d(np.asarray(column, dtype=np.float64))[:, None]
    return np.sum(f[None, :] * -np.expm1(-(k + kappa_c) * m), axis=1)


def _odf_task(args):
    (lines, species, abundance, T, lp, v, layout, opts, bins) = args
    steps, counters, _ = odf_point(lines, species, abundance, T, lp, v, layout, opts, bins)
    return steps, counters


def odf(lines, species, abundance, points, layout, opts, bins=None, workers=1):
    """ODF table out[point][bin][step] for every point (bins subset optional).

    With workers > 1 the points are handed out to a process pool.
    """
    tasks = [(lines, species, abundance, float(points.T_K[i]), float(points.log10_P[i]),
              float(points.vturb_kms[i]), layout, opts, bins) for i in range(points.n_points)]
    if workers > 1 and len(tasks) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            res = pool.map(_odf_task, tasks)
    else:
        res = [_odf_task(t) for t in tasks]
    out = np.stack([r[0] for r in res])
    counters = [r[1] for r in res]
    return out, counters

"""Shared helpers of the GPU tests: oracle-side ambiguity detection.

Where floating point decides an integer (a line kept or not, a window edge
rounded up or down) the HIP path and the oracle may take different, equally
valid decisions when the real value sits within rounding of the boundary.
These helpers find such cases from the oracle's real-valued decisions; a bin
that holds one is not skipped: its reference is recomputed by the oracle with
the GPU's own decisions, after checking that those differ from the oracle's
only at such ties (so they are valid), and compared at the same tolerance.
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


class Reach:
    """The lines whose window can reach given bins at one (T, v_turb).

    A window spans at most opts.window_cap_doppler Doppler widths, and the
    Doppler width b = sqrt(2 k T / m + v^2) / c is largest for the lightest
    species, so at most y = cap * b_max in relative frequency on either side
    of the centre: the window of a line at lambda_0 lies within
    [lambda_0 / (1 + y), lambda_0 / (1 - y)].  A line can then touch a bin
    whose points run from lambda_a to lambda_b only if
    lambda_a (1 - y) <= lambda_0 <= lambda_b (1 + y); the bound is widened
    by 0.1 % and a few grid steps for the window's integer rounding.  The
    subset is a superset of the lines the oracle needs for those bins, and
    much smaller than the whole list at cool points."""

    def __init__(self, lines, species, layout, opts):
        from oracle.constants import AMU
        lam = np.asarray(lines.lambda_nm)
        self.order = np.argsort(lam, kind="stable")
        self.lam = lam[self.order]
        self.m_min = float(np.min(species.mass_amu)) * AMU
        self.cap = float(opts.window_cap_doppler)
        self.layout = layout

    def y(self, T, vturb_kms):
        from oracle.constants import C_LIGHT, K_BOLTZ
        v = vturb_kms * 1e5
        b_max = math.sqrt(2.0 * K_BOLTZ * T / self.m_min + v * v) / C_LIGHT
        return self.cap * b_max * 1.001 + 1e-5

    def lines_for(self, bins, T, vturb_kms):
        """Sorted indices (into the list) of the lines that can reach the bins."""
        e = self.layout.bin_edges
        y = self.y(T, vturb_kms)
        parts = []
        for b in bins:
            l0 = float(oracle.grid_lambda_nm(self.layout, e[b]))
            l1 = float(oracle.grid_lambda_nm(self.layout, e[b + 1] - 1))
            i0 = np.searchsorted(self.lam, l0 * (1.0 - y), side="left")
            i1 = np.searchsorted(self.lam, l1 * (1.0 + y), side="right")
            parts.append(self.order[i0:i1])
        if not parts:
            return np.zeros(0, dtype=np.int64)
        return np.unique(np.concatenate(parts))


def floor_values(layout, opts, j0, j1):
    return opts.cutoff * oracle.physics.kappa_c(oracle.grid_lambda_nm(layout, np.arange(j0, j1)), opts)


def rel_err(got, ref):
    return np.abs(np.asarray(got, dtype=np.float64) / np.asarray(ref, dtype=np.float64) - 1.0)


def log10_err(got, ref):
    return np.abs(np.log10(np.asarray(got, dtype=np.float64)) - np.log10(np.asarray(ref, dtype=np.float64)))


def fmt(x):
    return f"{x:.3e}" if isinstance(x, float) and math.isfinite(x) else str(x)


def gpu_decisions(plan, abundance, points, i):
    """The GPU's survivors of point i and their integer windows, in the
    oracle's terms: sorted caller line indices with their (j_lo, j_hi)."""
    g = plan.stage_lines(abundance, points, point=i)
    order = np.argsort(g["orig"], kind="stable")
    return dict(orig=g["orig"][order], jlo=g["jlo"][order].astype(np.int64),
                jhi=g["jhi"][order].astype(np.int64))


def oracle_bin_with_gpu_decisions(lq, layout, opts, b, dec, sub_to_full=None):
    """The oracle's ODF steps of bin b computed with the GPU's keep and
    window decisions (dec from gpu_decisions) in place of its own.

    Every line whose window can reach the bin is checked first: the GPU may
    differ from the oracle only where floating point decides within
    rounding of a boundary (a keep test with |core/thr - 1| < KEEP_RTOL, or
    a window edge within EDGE_ATOL of an integer n, which is then n or n + 1
    at the start, n - 1 or n at the end), so the decisions taken are valid
    ones.  lq may cover a subset of the lines,
    sub_to_full mapping its entries to the caller's line indices."""
    e = np.asarray(layout.bin_edges, dtype=np.int64)
    j0, j1 = int(e[b]), int(e[b + 1])
    n = lq["S"].size
    full = np.arange(n) if sub_to_full is None else np.asarray(sub_to_full, dtype=np.int64)
    k = np.searchsorted(dec["orig"], full)
    kc = np.minimum(k, max(dec["orig"].size - 1, 0))
    gsurv = (k < dec["orig"].size) & (dec["orig"][kc] == full) if dec["orig"].size else np.zeros(n, bool)
    gjlo = np.where(gsurv, dec["jlo"][kc] if dec["orig"].size else 0, lq["jlo"])
    gjhi = np.where(gsurv, dec["jhi"][kc] if dec["orig"].size else 0, lq["jhi"])
    osurv = lq["surv"]
    reach = ((osurv & (lq["jlo"] <= j1) & (lq["jhi"] >= j0 - 1))
             | (gsurv & (gjlo <= j1) & (gjhi >= j0 - 1)))
    keep_tie, lo_tie, hi_tie = ambiguous_lines(lq)
    both = osurv & gsurv
    bad_keep = reach & (osurv != gsurv) & ~keep_tie & ~lo_tie & ~hi_tie
    # a start edge ceil(j_lo_r) with j_lo_r within rounding of an integer n
    # is n or n + 1; an end edge floor(j_hi_r) is n - 1 or n (both clipped
    # to the grid as the window is)
    N = int(lq["N"])
    nlo = np.round(lq["jlo_r"])
    nhi = np.round(lq["jhi_r"])
    lo_ok = lo_tie & ((gjlo == np.maximum(nlo, 0)) | (gjlo == np.maximum(nlo + 1, 0)))
    hi_ok = hi_tie & ((gjhi == np.minimum(nhi, N - 1)) | (gjhi == np.minimum(nhi - 1, N - 1)))
    bad_lo = reach & both & (gjlo != lq["jlo"]) & ~lo_ok
    bad_hi = reach & both & (gjhi != lq["jhi"]) & ~hi_ok
    assert not bad_keep.any(), f"GPU keep decisions differ from the oracle's away from a tie: {np.nonzero(bad_keep)[0][:5]}"
    assert not bad_lo.any(), f"GPU window starts differ away from a tie: {np.nonzero(bad_lo)[0][:5]}"
    assert not bad_hi.any(), f"GPU window ends differ away from a tie: {np.nonzero(bad_hi)[0][:5]}"
    lq2 = dict(lq)
    lq2["surv"] = np.where(reach, gsurv, osurv)
    lq2["jlo"] = np.where(reach & gsurv, gjlo, lq["jlo"])
    lq2["jhi"] = np.where(reach & gsurv, gjhi, lq["jhi"])
    kl = oracle.fine_opacity(lq2, layout, j0, j1)
    kt = np.maximum(kl, floor_values(layout, opts, j0, j1))
    return oracle.odf_reduce_bin(kt, layout.step_frac, opts.mean)


def compare_points(w, out, prec, bins=None, abundance=None, plan=None):
    """Largest relative and log10 errors of out[point][bin][step] against the
    oracle's ODF over every bin, and the number of bins whose reference was
    computed with the GPU's own keep and window decisions (bins that hold a
    near-tie decision; plan must then be the live plan that computed out)."""
    a = w.species.abundance if abundance is None else abundance
    worst, worst_log, resolved = 0.0, 0.0, 0
    for i in range(w.points.n_points):
        ref, _, ex = oracle.odf_point(w.lines, w.species, a, float(w.points.T_K[i]),
                                      float(w.points.log10_P[i]), float(w.points.vturb_kms[i]),
                                      w.layout, w.options, bins)
        bsel = np.arange(w.layout.n_bins) if bins is None else np.asarray(bins)
        amb = ambiguous_bins(ex["lq"], w.layout.bin_edges)
        got = out[i][bsel]
        dec = None
        for k, b in enumerate(bsel):
            r = ref[k]
            if int(b) in amb:
                assert plan is not None, "a bin with a near-tie decision needs the live plan"
                if dec is None:
                    dec = gpu_decisions(plan, a, w.points, i)
                r = oracle_bin_with_gpu_decisions(ex["lq"], w.layout, w.options, int(b), dec)
                resolved += 1
            worst = max(worst, float(rel_err(got[k], r).max()))
            worst_log = max(worst_log, float(log10_err(got[k], r).max()))
    return worst, worst_log, resolved

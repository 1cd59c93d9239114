"""Seeded synthetic workloads for ODF generation (inputs only, no physics).

This module is shared by the FP64 CPU oracle and the HIP path, so it holds
none of the method's arithmetic: it draws line lists, species tables, T-P-v
point grids and bin layouts with numpy's PCG64 generator and returns plain
arrays.  The shapes follow the paper's workloads: a DFSYNTHE-style T-P grid
of 57 temperatures by 25 pressures spanning 12 decades in P (Sec. 4.2), a
high-resolution grid at R = 500 000 starting at 8.9766 nm (App. E, grid
formula), twelve sub-bins (Sec. 2.3 and Sec. 4.1) and line lists of 1e7-1e8
entries standing in for the Kurucz/VALD lists (Sec. 2.3, Sec. 4.4), which are
not available here.

Draw order for a seed: species table, then lines, then requests.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

#: grid start of the paper's high-resolution grid [nm] (App. E)
LAMBDA_FIRST_FULL_NM = 8.9766
#: grid end [nm] (App. E)
LAMBDA_LAST_FULL_NM = 10000.0
#: resolving power of the high-resolution grid (App. E)
RESOLVING_POWER = 500000.0
#: sub-bin fractions, lowest opacity first: nine of 10 %, then 5 %, 4 %, 1 %
STEP_FRAC_12 = np.array([0.1] * 9 + [0.05, 0.04, 0.01], dtype=np.float64)


@dataclass
class Species:
    mass_amu: np.ndarray      # [S] f64
    chi_ev: np.ndarray        # [S, K-1] f64 ionisation energies
    part_fn: np.ndarray       # [S, K] f64 constant partition functions
    abundance: np.ndarray     # [S] f64 N_s / N_H
    alpha: np.ndarray         # [S] bool, alpha-element flag

    @property
    def n_species(self) -> int:
        return int(self.mass_amu.shape[0])

    @property
    def n_stages(self) -> int:
        return int(self.part_fn.shape[1])


@dataclass
class Lines:
    lambda_nm: np.ndarray     # [L] f64 vacuum wavelength
    log_gf: np.ndarray        # [L] f64
    e_low_ev: np.ndarray      # [L] f64 lower-level energy
    species: np.ndarray       # [L] i32
    stage: np.ndarray         # [L] i32 (0 = neutral)
    log_g_rad: np.ndarray     # [L] f64 log10 gamma_rad [s^-1]
    log_g_stark: np.ndarray   # [L] f64 log10 gamma_Stark per electron [s^-1 cm^3]
    log_g_vdw: np.ndarray     # [L] f64 log10 gamma_vdW per heavy particle [s^-1 cm^3]

    @property
    def n_lines(self) -> int:
        return int(self.lambda_nm.shape[0])

    def take(self, idx) -> "Lines":
        return Lines(*(getattr(self, f)[idx] for f in _LINE_FIELDS))


_LINE_FIELDS = ("lambda_nm", "log_gf", "e_low_ev", "species", "stage",
                "log_g_rad", "log_g_stark", "log_g_vdw")


@dataclass
class Layout:
    lambda_first_nm: float
    lambda_last_nm: float
    resolving_power: float
    bin_edges: np.ndarray     # [n_bins+1] i64 fine-grid indices
    step_frac: np.ndarray     # [n_steps] f64, lowest opacity first

    @property
    def n_bins(self) -> int:
        return int(self.bin_edges.shape[0] - 1)

    @property
    def n_steps(self) -> int:
        return int(self.step_frac.shape[0])


@dataclass
class Points:
    T_K: np.ndarray
    log10_P: np.ndarray
    vturb_kms: np.ndarray

    @property
    def n_points(self) -> int:
        return int(self.T_K.shape[0])

    def take(self, idx) -> "Points":
        return Points(self.T_K[idx], self.log10_P[idx], self.vturb_kms[idx])


@dataclass
class Options:
    precision: str = "fp64"         # "fp64" | "mixed"
    mean: str = "geometric"         # "geometric" | "arithmetic"
    cutoff: float = 1e-4
    window_cap_doppler: float = 500.0
    pe_over_p: float = 0.1
    kappa_c_ref: float = 1.0        # cm^2 / g at lambda_c_ref
    lambda_c_ref_nm: float = 500.0
    kappa_c_power: float = 3.0
    output: str = "table"           # "table" (ODF) | "fine" (pre-tabulated opacity per fine point)
    electrons: str = "fixed"        # "fixed" (P_e = pe_over_p P) | "equilibrium" (ionisation equilibrium)


@dataclass
class Request:
    abundance: np.ndarray
    points: Points
    arrival_s: float = 0.0


@dataclass
class Workload:
    name: str
    species: Species
    lines: Lines
    layout: Layout
    points: Points
    options: Options = field(default_factory=Options)
    requests: list = field(default_factory=list)


def grid_size(lambda_first_nm: float, lambda_last_nm: float, resolving_power: float) -> int:
    """Number of fine points with lambda_first * q^j <= lambda_last, q = 1 + 1/R.

    Input construction only (a bin layout must end inside the grid).  The
    count is taken in 60-digit decimal arithmetic so that it does not depend
    on binary rounding at the grid end.
    """
    import decimal
    ctx = decimal.Context(prec=60)
    lf = decimal.Decimal(repr(float(lambda_first_nm)))
    ll = decimal.Decimal(repr(float(lambda_last_nm)))
    lq = ctx.ln(decimal.Decimal(1) + ctx.divide(decimal.Decimal(1), decimal.Decimal(repr(float(resolving_power)))))
    ratio = ctx.ln(ctx.divide(ll, lf))
    return int(ctx.divide(ratio, lq).to_integral_value(rounding=decimal.ROUND_FLOOR)) + 1


def equal_bins(n_fine: int, n_bins: int) -> np.ndarray:
    return np.array([(b * n_fine) // n_bins for b in range(n_bins + 1)], dtype=np.int64)


def ramp_bins(n_fine: int, n_bins: int, w0: float = 500.0) -> np.ndarray:
    """Geometric ramp of bin widths w_b = w0 * r^b with r chosen so that the
    widths sum to n_fine; edges are the floors of the cumulative sums."""
    target = float(n_fine)

    def total(r):
        return w0 * (r ** n_bins - 1.0) / (r - 1.0)

    lo, hi = 1.0 + 1e-12, 1.1
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if total(mid) < target:
            lo = mid
        else:
            hi = mid
    r = 0.5 * (lo + hi)
    widths = w0 * r ** np.arange(n_bins, dtype=np.float64)
    edges = np.zeros(n_bins + 1, dtype=np.int64)
    edges[1:] = np.floor(np.cumsum(widths)).astype(np.int64)
    edges[-1] = n_fine
    return edges


def draw_species(rng: np.random.Generator, n_species: int, n_stages: int) -> Species:
    mass = rng.uniform(12.0, 60.0, n_species)
    chi = np.zeros((n_species, max(n_stages - 1, 0)))
    if n_stages >= 2:
        chi[:, 0] = rng.uniform(6.0, 14.0, n_species)
    for k in range(1, n_stages - 1):
        chi[:, k] = chi[:, k - 1] + rng.uniform(6.0, 14.0, n_species)
    part = rng.uniform(1.0, 30.0, (n_species, n_stages))
    abund = 10.0 ** rng.uniform(-12.0, -4.0, n_species)
    alpha = (np.arange(n_species) % 4) == 0
    return Species(mass, chi, part, abund, alpha)


def draw_lines(rng: np.random.Generator, n_lines: int, n_species: int, n_stages: int,
               lam_lo: float, lam_hi: float, log_uniform: bool) -> Lines:
    if log_uniform:
        lam = np.exp(rng.uniform(math.log(lam_lo), math.log(lam_hi), n_lines))
    else:
        lam = rng.uniform(lam_lo, lam_hi, n_lines)
    log_gf = rng.uniform(-5.0, 0.5, n_lines)
    e_low = rng.uniform(0.0, 10.0, n_lines)
    ss = rng.integers(0, n_species * n_stages, n_lines)
    species = (ss // n_stages).astype(np.int32)
    stage = (ss % n_stages).astype(np.int32)
    g_rad = rng.normal(8.0, 0.5, n_lines)
    g_stark = rng.normal(-5.0, 0.5, n_lines)
    g_vdw = rng.normal(-7.5, 0.5, n_lines)
    return Lines(lam, log_gf, e_low, species, stage, g_rad, g_stark, g_vdw)


def dfsynthe_tp_grid(vturbs=(2.0,)) -> Points:
    """57 temperatures log-spaced 2000..200000 K by 25 log10 P from -4 to 8
    (Sec. 4.2: 57 x 25 points, 12 decades in P), repeated per microturbulence."""
    T = 2000.0 * 100.0 ** (np.arange(57) / 56.0)
    lp = -4.0 + 0.5 * np.arange(25)
    TT, PP, VV = np.meshgrid(T, lp, np.asarray(vturbs, dtype=np.float64), indexing="ij")
    # order: vturb outermost, then T, then P (P fastest)
    TT = np.transpose(TT, (2, 0, 1)).ravel()
    PP = np.transpose(PP, (2, 0, 1)).ravel()
    VV = np.transpose(VV, (2, 0, 1)).ravel()
    return Points(TT.astype(np.float64), PP.astype(np.float64), VV.astype(np.float64))


def composition(species: Species, m_h: float, alpha_fe: float) -> np.ndarray:
    """Abundances scaled by metallicity [M/H] and alpha enhancement."""
    a = species.abundance * 10.0 ** m_h
    return np.where(species.alpha, a * 10.0 ** alpha_fe, a)


def config(idx: int, n_lines: int | None = None, n_requests: int | None = None,
           lam_range: tuple | None = None, n_bins: int | None = None) -> Workload:
    """Synthetic workload `idx` (1..5).

    1: one point, 1e4 lines in 300-310 nm, 5 species x 2 stages, 20 equal bins.
    2: 57 x 25 T-P grid, vturb 2 km/s, 1e7 lines 9 nm-10 um, 40 x 2, 1212 ramp bins.
    3: grid of 2 at vturb {0,1,2,4,8} km/s (mixed precision).
    4: Poisson request stream over 2's lines and bins ([M/H], [alpha/Fe] per request).
    5: 1e8 lines, 80 x 3, requests of the full grid at five vturb, bursts of 8.

    `n_lines`, `lam_range` (nm, nm) and `n_bins` shrink a configuration for
    tests; the draws keep their order so a shrunk config is self-consistent.
    """
    rng = np.random.default_rng(idx)
    opts = Options()
    if idx == 1:
        S, K = 5, 2
        sp = draw_species(rng, S, K)
        L = 10_000 if n_lines is None else n_lines
        lo, hi = lam_range if lam_range else (300.0, 310.0)
        lines = draw_lines(rng, L, S, K, lo, hi, log_uniform=False)
        lf, ll = 300.0, 310.0
        if lam_range:
            lf, ll = lam_range
        N = grid_size(lf, ll, RESOLVING_POWER)
        layout = Layout(lf, ll, RESOLVING_POWER, equal_bins(N, n_bins or 20), STEP_FRAC_12.copy())
        pts = Points(np.array([5000.0]), np.array([4.0]), np.array([2.0]))
        return Workload("cfg1", sp, lines, layout, pts, opts)
    if idx in (2, 3, 4):
        S, K = 40, 2
        L = 10_000_000
    elif idx == 5:
        S, K = 80, 3
        L = 100_000_000
    else:
        raise ValueError(f"unknown config {idx}")
    if n_lines is not None:
        L = n_lines
    sp = draw_species(rng, S, K)
    lf, ll = (LAMBDA_FIRST_FULL_NM, LAMBDA_LAST_FULL_NM)
    if lam_range:
        lf, ll = lam_range
    lines = draw_lines(rng, L, S, K, max(9.0, lf), ll, log_uniform=True)
    N = grid_size(lf, ll, RESOLVING_POWER)
    nb = 1212 if n_bins is None else n_bins
    edges = ramp_bins(N, nb) if (n_bins is None and lam_range is None) else equal_bins(N, nb)
    layout = Layout(lf, ll, RESOLVING_POWER, edges, STEP_FRAC_12.copy())
    if idx == 2:
        pts = dfsynthe_tp_grid((2.0,))
    elif idx == 3:
        pts = dfsynthe_tp_grid((0.0, 1.0, 2.0, 4.0, 8.0))
        opts = replace(opts, precision="mixed")
    elif idx == 4:
        pts = dfsynthe_tp_grid((2.0,))
        opts = replace(opts, precision="mixed")
    else:
        pts = dfsynthe_tp_grid((0.0, 1.0, 2.0, 4.0, 8.0))
        opts = replace(opts, precision="mixed")
    w = Workload(f"cfg{idx}", sp, lines, layout, pts, opts)
    if idx == 4:
        w.requests = draw_requests_cfg4(idx, sp, pts, 256 if n_requests is None else n_requests)
    elif idx == 5:
        w.requests = draw_requests_cfg5(idx, sp, pts, 32 if n_requests is None else n_requests)
    return w


def draw_requests_cfg4(seed: int, sp: Species, grid: Points, n: int, rate_hz: float = 20.0):
    """Poisson stream; each request has its own composition and a random
    subset of 1..1425 distinct (T, P) points at vturb 2 km/s."""
    reqs = []
    t = 0.0
    for rid in range(n):
        r = np.random.default_rng(seed * 1_000_003 + rid)
        t += r.exponential(1.0 / rate_hz)
        m_h = r.uniform(-2.0, 0.5)
        a_fe = r.uniform(0.0, 0.4)
        npts = int(r.integers(1, grid.n_points + 1))
        idx = np.sort(r.choice(grid.n_points, npts, replace=False))
        reqs.append(Request(composition(sp, m_h, a_fe), grid.take(idx), t))
    return reqs


def draw_requests_cfg5(seed: int, sp: Species, grid: Points, n: int,
                       burst_rate_hz: float = 5.0 / 8.0, burst: int = 8):
    """Bursts of 8 requests, burst arrivals Poisson so the mean request rate
    is 5/s; each request covers the whole grid at five vturb values."""
    reqs = []
    t = 0.0
    rid = 0
    while rid < n:
        r = np.random.default_rng(seed * 1_000_003 + rid)
        t += r.exponential(1.0 / burst_rate_hz)
        for _ in range(min(burst, n - rid)):
            rr = np.random.default_rng(seed * 1_000_003 + rid)
            m_h = rr.uniform(-2.0, 0.5)
            a_fe = rr.uniform(0.0, 0.4)
            reqs.append(Request(composition(sp, m_h, a_fe), grid, t))
            rid += 1
    return reqs


def small_points(T, logP, v) -> Points:
    return Points(np.atleast_1d(np.asarray(T, dtype=np.float64)),
                  np.atleast_1d(np.asarray(logP, dtype=np.float64)),
                  np.atleast_1d(np.asarray(v, dtype=np.float64)))

"""Populations, line strengths, pre-selection and windows.  TEST INFRASTRUCTURE ONLY.

Every quantity is FP64 and follows the paper's statement:

* point state and Saha-Boltzmann stage populations N_k/U_k per gram
  (Sec. 2.1; App. A; App. E first stage, item i), with the electron pressure
  either fixed at a given fraction of the gas pressure or found from the
  ionisation equilibrium of App. A (without molecules): the conservation
  equations written in the neutral densities and n_e, solved by
  Newton-Raphson with a dense LU ("triangular decomposition") of the
  Jacobian until every relative change is below 1e-4;
* Doppler width dnu_D = (nu_0/c) sqrt(2kT/m + v_turb^2) (App. E, equation for
  dnu_D);
* line absorption coefficient per gram (Sec. 2.1, eq. l_nu_line), written as
  ell = S * H(x, a) with S = (sqrt(pi) e^2 / m_e c) g f (N_k/U_k)/rho
  e^{-E/kT} (1 - e^{-h nu_0/kT}) / dnu_D, x = (nu - nu_0)/dnu_D and
  a = gamma / (4 pi dnu_D);
* pre-selection of lines whose core opacity falls below cutoff * kappa_c
  (Sec. 4.3; App. E selection conditions), taken per line;
* the profile window in which a kept line is summed onto the grid.
"""
import math

import numpy as np
from scipy.special import erfcx

from .constants import (AMU, C_LIGHT, CHI_HYDROGEN_EV, EV, HC_K_NM, K_BOLTZ,
                        M_HYDROGEN_AMU, PI_E2_MC, SAHA_CONST, U_HYDROGEN)


def point_state(T, log10_P, pe_over_p, abundance, mass_amu, n_e=None):
    """Electron density, heavy-particle density, H density and mass density.

    P_e = pe_over_p * P, n_e = P_e / kT, and heavy particles (every atom and
    ion) N_h = (P - P_e)/kT; or, given n_e, N_h = P/kT - n_e.  N_h is split
    over H and the metals by the abundances N_s/N_H; rho counts H with
    1.008 amu and each metal with its mass.
    """
    P = 10.0 ** log10_P
    kT = K_BOLTZ * T
    if n_e is None:
        pe = pe_over_p * P
        n_e = pe / kT
        n_heavy = (P - pe) / kT
    else:
        n_heavy = P / kT - n_e
    n_H = n_heavy / (1.0 + np.sum(abundance))
    rho = n_H * AMU * (M_HYDROGEN_AMU + np.sum(abundance * mass_amu))
    return dict(T=T, P=P, n_e=n_e, n_heavy=n_heavy, n_H=n_H, rho=rho)


def stage_fractions(T, n_e, chi_ev, part_fn):
    """Ionisation-stage fractions f[s, k] from the Saha equation.

    N_{k+1} n_e / N_k = 2 (U_{k+1}/U_k) (2 pi m_e k T / h^2)^{3/2}
    e^{-chi_k / kT}; the ratios are chained in log space and normalised so
    that the stages of each species sum to one.
    """
    S, K = part_fn.shape
    logf = np.zeros((S, K))
    for k in range(K - 1):
        ln_r = (math.log(2.0) + np.log(part_fn[:, k + 1]) - np.log(part_fn[:, k])
                + math.log(SAHA_CONST) + 1.5 * math.log(T)
                - chi_ev[:, k] * EV / (K_BOLTZ * T) - math.log(n_e))
        logf[:, k + 1] = logf[:, k] + ln_r
    m = logf.max(axis=1, keepdims=True)
    lse = m + np.log(np.sum(np.exp(logf - m), axis=1, keepdims=True))
    return np.exp(logf - lse)


def saha_ratios(T, chi_ev, part_fn):
    """Phi[i, k] = n_{k+1} n_e / n_k = 2 (U_{k+1}/U_k) (2 pi m_e k T/h^2)^{3/2}
    e^{-chi_k/kT} (Sec. 2.1, Saha-Boltzmann)."""
    U = np.asarray(part_fn, dtype=np.float64)
    chi = np.asarray(chi_ev, dtype=np.float64)
    return (2.0 * U[:, 1:] / U[:, :-1] * SAHA_CONST * T ** 1.5
            * np.exp(-chi * EV / (K_BOLTZ * T)))


def equilibrium_elements(abundance, chi_ev, part_fn):
    """Elements of the ionisation equilibrium: hydrogen (two stages, row 0)
    followed by every species of the table; stages missing from hydrogen are
    given zero weight by an infinite ionisation energy."""
    S, K = np.asarray(part_fn).shape
    K = max(K, 2)
    chi = np.full((S + 1, K - 1), np.inf)
    U = np.ones((S + 1, K))
    chi[0, 0] = CHI_HYDROGEN_EV
    U[0, :2] = U_HYDROGEN
    if S:
        chi[1:, :np.asarray(chi_ev).shape[1]] = chi_ev
        U[1:, :np.asarray(part_fn).shape[1]] = part_fn
    A = np.concatenate([[1.0], np.asarray(abundance, dtype=np.float64)])
    return A, chi, U


def _element_sums(R, ne):
    """G_i, Q_i and their derivatives in n_e (see ionisation_equilibrium)."""
    kk = np.arange(R.shape[1], dtype=np.float64)
    p = ne ** -kk
    G = R @ p
    Q = R @ (kk * p)
    return G, Q, -Q / ne, -(R @ (kk * kk * p)) / ne


def equilibrium_system(x, R, A, n_tot):
    """Residuals f and Jacobian M = df/dx of the equilibrium equations at
    x = (neutral densities of the elements, n_e); R[i, k] the products of the
    Saha ratios, A the abundances by number relative to hydrogen (A[0] = 1)."""
    E = R.shape[0]
    n, ne = x[:E], x[E]
    G, Q, dG, dQ = _element_sums(R, ne)
    f = np.empty(E + 1)
    f[0] = np.sum(n * G) + ne - n_tot
    f[1:E] = n[1:] * G[1:] - A[1:] * n[0] * G[0]
    f[E] = np.sum(n * Q) - ne
    M = np.zeros((E + 1, E + 1))
    M[0, :E] = G
    M[0, E] = np.sum(n * dG) + 1.0
    for s in range(1, E):
        M[s, 0] = -A[s] * G[0]
        M[s, s] = G[s]
        M[s, E] = n[s] * dG[s] - A[s] * n[0] * dG[0]
    M[E, :E] = Q
    M[E, E] = np.sum(n * dQ) - 1.0
    return f, M


def ionisation_equilibrium(T, log10_P, abundance, chi_ev, part_fn, tol=1e-4, max_iter=100):
    """Electron density from the ionisation equilibrium of App. A (no molecules).

    Unknowns: the neutral densities n_i of hydrogen and of every species and
    the electron density n_e.  With R[i, k] = prod_{m<k} Phi[i, m] an element
    holds N_i = n_i G_i, G_i = sum_k R[i, k] n_e^-k, and gives Q_i n_i
    electrons, Q_i = sum_k k R[i, k] n_e^-k.  The equations are
      particles:  sum_i n_i G_i + n_e - P/kT = 0
      abundance:  n_s G_s - A_s n_H G_H = 0        (each species s)
      charge:     sum_i n_i Q_i - n_e = 0.
    Newton-Raphson: M dn = f with M the Jacobian (a dense LU solve), then
    n <- n - lam dn, where lam <= 1 keeps every unknown within a factor of 10
    of its value; stop when every |lam dn_i| / n_i < tol.
    Start: n_e = min(sqrt(sum_i nu_i P/kT Phi[i, 0]), P/2kT) (the weak-
    ionisation limit, capped at full ionisation of hydrogen) and the neutral
    densities that satisfy the particle and abundance equations for it.
    Returns dict(n_e, n_neutral, iterations, converged).
    """
    A, chi, U = equilibrium_elements(abundance, chi_ev, part_fn)
    E, K = U.shape
    kT = K_BOLTZ * T
    n_tot = 10.0 ** log10_P / kT
    Phi = saha_ratios(T, chi, U)
    R = np.ones((E, K))
    for k in range(1, K):
        R[:, k] = R[:, k - 1] * Phi[:, k - 1]
    nu = A / np.sum(A)
    ne = min(math.sqrt(n_tot * np.sum(nu * Phi[:, 0])), 0.5 * n_tot)
    G = _element_sums(R, ne)[0]
    x = np.concatenate([nu * (n_tot - ne) / G, [ne]])
    it = 0
    converged = False
    while it < max_iter:
        it += 1
        f, M = equilibrium_system(x, R, A, n_tot)
        dx = np.linalg.solve(M, f)
        lam = 1.0
        for xi, di in zip(x, dx):
            if di > 0.0:
                lam = min(lam, 0.9 * xi / di)
            elif di < 0.0:
                lam = min(lam, 9.0 * xi / -di)
        x = x - lam * dx
        if np.max(np.abs(lam * dx) / x) < tol:
            converged = True
            break
    return dict(n_e=float(x[E]), n_neutral=x[:E].copy(), iterations=it, converged=converged)


def electron_density(T, log10_P, abundance, species, opts):
    """n_e of a point: fixed P_e / P, or the ionisation equilibrium."""
    if getattr(opts, "electrons", "fixed") == "equilibrium":
        r = ionisation_equilibrium(T, log10_P, abundance, species.chi_ev, species.part_fn)
        if not r["converged"]:
            raise RuntimeError(f"ionisation equilibrium did not converge at T={T}, log P={log10_P}")
        return r["n_e"]
    return opts.pe_over_p * 10.0 ** log10_P / (K_BOLTZ * T)


def populations(state, abundance, chi_ev, part_fn):
    """N_k / (U_k rho) per species and stage, in g^-1 (App. E, item i)."""
    f = stage_fractions(state["T"], state["n_e"], chi_ev, part_fn)
    return abundance[:, None] * state["n_H"] * f / (part_fn * state["rho"])


def kappa_c(lambda_nm, opts):
    """Synthetic continuum opacity kappa_ref (lambda/lambda_ref)^power [cm^2/g]."""
    return opts.kappa_c_ref * (np.asarray(lambda_nm) / opts.lambda_c_ref_nm) ** opts.kappa_c_power


def line_quantities(lines, species, abundance, T, log10_P, vturb_kms, layout, opts):
    """Per-line S, a, b, keep decision and window for one (T, P, v) point.

    Returns a dict of arrays over all lines (input order):
      S      line strength [cm^2 g^-1] so that ell = S * H(x, a)
      a      damping parameter gamma / (4 pi dnu_D)
      b      dnu_D / nu_0
      thr    cutoff * kappa_c(lambda_0)
      core   S * H(0, a), the line-core opacity used by the selection
      keep   core >= thr
      xw     half-window in Doppler widths (capped)
      jstar  fractional grid index of the line centre
      jlo_r, jhi_r  real-valued window edges before ceil / floor
      jlo, jhi      integer window clipped to the grid
      surv   kept with a non-empty clipped window
    """
    n_e = electron_density(T, log10_P, abundance, species, opts)
    st = point_state(T, log10_P, opts.pe_over_p, abundance, species.mass_amu, n_e=n_e)
    pop = populations(st, abundance, species.chi_ev, species.part_fn)
    kT = K_BOLTZ * T
    lam = lines.lambda_nm
    nu0 = C_LIGHT / (lam * 1e-7)
    m = species.mass_amu[lines.species] * AMU
    v = vturb_kms * 1e5
    b = np.sqrt(2.0 * kT / m + v * v) / C_LIGHT
    dnu_d = b * nu0
    stim = -np.expm1(-HC_K_NM / (lam * T))
    boltz = np.exp(-lines.e_low_ev * EV / kT)
    p = pop[lines.species, lines.stage]
    S = PI_E2_MC * 10.0 ** lines.log_gf * p * boltz * stim / (math.sqrt(math.pi) * dnu_d)
    t4 = T / 1.0e4
    gamma = (10.0 ** lines.log_g_rad
             + 10.0 ** lines.log_g_stark * st["n_e"] * t4 ** (1.0 / 6.0)
             + 10.0 ** lines.log_g_vdw * st["n_heavy"] * t4 ** 0.3)
    a = gamma / (4.0 * math.pi * dnu_d)
    thr = opts.cutoff * kappa_c(lam, opts)
    core = S * erfcx(a)
    keep = core >= thr
    # half-window: both envelope terms (Gaussian core and Lorentz wing)
    # fall to thr/2 or below beyond xw; capped at window_cap_doppler
    with np.errstate(divide="ignore", invalid="ignore"):
        xg = np.sqrt(np.maximum(0.0, np.log(2.0 * S / thr)))
        xl = np.sqrt(2.0 * S * a / (math.sqrt(math.pi) * thr))
    xw = np.minimum(opts.window_cap_doppler, np.maximum(xg, xl))
    lnq = math.log1p(1.0 / layout.resolving_power)
    jstar = np.log(lam / layout.lambda_first_nm) / lnq
    jlo_r = jstar - np.log1p(xw * b) / lnq
    jhi_r = jstar - np.log1p(-xw * b) / lnq
    N = grid_size(layout.lambda_first_nm, layout.lambda_last_nm, layout.resolving_power)
    jlo = np.maximum(np.ceil(jlo_r), 0).astype(np.int64)
    jhi = np.minimum(np.floor(jhi_r), N - 1).astype(np.int64)
    surv = keep & (jlo <= jhi)
    return dict(state=st, pop=pop, S=S, a=a, b=b, thr=thr, core=core, keep=keep,
                xw=xw, jstar=jstar, jlo_r=jlo_r, jhi_r=jhi_r, jlo=jlo, jhi=jhi,
                surv=surv, gamma=gamma, N=N)


def grid_size(lambda_first_nm, lambda_last_nm, resolving_power):
    """N = floor(ln(lambda_last/lambda_first) / ln q) + 1 with q = 1 + 1/R
    (App. E grid formula lambda_n = lambda_1 q^(n-1))."""
    lnq = math.log1p(1.0 / resolving_power)
    return int(math.floor(math.log(lambda_last_nm / lambda_first_nm) / lnq)) + 1

// Line-list preparation, per-point state, line pre-selection and survivor
// compaction (gfx950).
//
// Physics (Witzke et al. 2021):
//  - Saha-Boltzmann stage populations N_k/U_k per gram with the electron
//    density fixed by P_e = pe_over_p * P or taken from the ionisation
//    equilibrium of hydrogen and every species (Sec. 2.1; App. A; App. E
//    first stage item i).
//  - Doppler width dnu_D = (nu0/c) sqrt(2kT/m + v_turb^2) (App. E).
//  - Line strength S of ell_nu = S H(x, a) from eq. l_nu_line (Sec. 2.1),
//    damping parameter a = gamma / (4 pi dnu_D).
//  - Pre-selection: keep a line when its core opacity S H(0, a) reaches
//    cutoff * kappa_c(lambda0) (Sec. 4.3; App. E selection conditions).
//  - Window: half-width where the Gaussian and Lorentz envelopes of the
//    profile fall to half the cut, capped in Doppler widths.
// All of this is FP64: the Boltzmann and Saha factors span more than the
// FP32 range at the cool end of the grid.
#include "odf_internal.h"

namespace odf {

__global__ void k_prep_lines(int64_t n, const double* __restrict__ lam_nm,
                             const double* __restrict__ log_gf, const double* __restrict__ e_ev,
                             const double* __restrict__ lg_rad, const double* __restrict__ lg_stark,
                             const double* __restrict__ lg_vdw, const int32_t* __restrict__ species,
                             const int32_t* __restrict__ stage, int32_t n_stages,
                             double lambda_first_nm, double lnq, double cutoff, double kc_ref,
                             double kc_lref, double kc_pow, double* j0s, double* amp, double* e_k,
                             double* hc_k, double* g_rad, double* g_stark, double* g_vdw,
                             double* thr, int32_t* ss) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lam = lam_nm[i];
  const double nu0 = kC / (lam * 1e-7);
  const double pi_e2_mc = kPi * kEcharge * kEcharge / (kMe * kC);
  j0s[i] = log(lam / lambda_first_nm) / lnq;
  amp[i] = pi_e2_mc * exp10(log_gf[i]) / (kSqrtPi * nu0);
  e_k[i] = e_ev[i] * kEv / kK;
  hc_k[i] = kH * kC / kK * 1e7 / lam;
  const double four_pi_nu0 = 4.0 * kPi * nu0;
  g_rad[i] = exp10(lg_rad[i]) / four_pi_nu0;
  g_stark[i] = exp10(lg_stark[i]) / four_pi_nu0;
  g_vdw[i] = exp10(lg_vdw[i]) / four_pi_nu0;
  thr[i] = cutoff * kc_ref * pow(lam / kc_lref, kc_pow);
  ss[i] = species[i] * n_stages + stage[i];
}

hipError_t launch_prep_lines(hipStream_t st, int64_t n, const double* lam_nm, const double* log_gf,
                             const double* e_ev, const double* lg_rad, const double* lg_stark,
                             const double* lg_vdw, const int32_t* species, const int32_t* stage,
                             int32_t n_stages, double lambda_first_nm, double lnq, double cutoff,
                             double kc_ref, double kc_lref, double kc_pow, double* j0s, double* amp,
                             double* e_k, double* hc_k, double* g_rad, double* g_stark,
                             double* g_vdw, double* thr, int32_t* ss) {
  if (n == 0) return hipSuccess;
  const int64_t nb = (n + 255) / 256;
  hipLaunchKernelGGL(k_prep_lines, dim3((unsigned)nb), dim3(256), 0, st, n, lam_nm, log_gf, e_ev,
                     lg_rad, lg_stark, lg_vdw, species, stage, n_stages, lambda_first_nm, lnq,
                     cutoff, kc_ref, kc_lref, kc_pow, j0s, amp, e_k, hc_k, g_rad, g_stark, g_vdw,
                     thr, ss);
  return hipGetLastError();
}

// ---- ionisation equilibrium (App. A, without molecules) --------------------
//
// Elements: hydrogen (two stages) and every species of the table.  With the
// Saha ratios phi_k = n_{k+1} n_e / n_k, R_k = phi_0 ... phi_{k-1}, an
// element of neutral density n holds N = n G nuclei and gives n Q
// electrons, G = sum_k R_k n_e^-k, Q = sum_k k R_k n_e^-k.  Unknowns: the
// neutral densities and n_e; equations: particles (sum N + n_e = P/kT),
// abundances (N_s = A_s N_H) and charge (sum n Q = n_e).  Each Newton step
// solves J d = f.  J has nonzeros only in the hydrogen column, the n_e
// column, the particle row and the charge row, so eliminating every
// species' own unknown leaves a 2x2 system in (d_H, d_e): O(S) work per
// step, one species per lane, with wave sums.  The step is scaled by the
// largest lam <= 1 that keeps every unknown within a factor of 10 of its
// value; the iteration stops when every relative change is below 1e-4.
// Start: n_e = min(sqrt(P/kT sum nu_i phi_0,i), P/2kT) (weak ionisation,
// capped at fully ionised hydrogen), neutral densities consistent with it.
constexpr double kChiH = 13.598434599702;   // eV, H I
constexpr double kU_HI = 2.0, kU_HII = 1.0;
constexpr double kNeTol = 1e-4;

// Butterfly reductions over the 64 lanes: every lane ends with the same
// bits (each step adds the same two values in both lanes).
__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// G, Q and their n_e derivatives from the Saha ratios phi[0..K-2].
struct ElemGQ {
  double G, Q, dG, dQ;
};
__device__ __forceinline__ ElemGQ elem_gq(const double* phi, int K, double inv_ne) {
  ElemGQ e{1.0, 0.0, 0.0, 0.0};
  double R = 1.0, q2 = 0.0;
  double pk = 1.0;
  for (int k = 1; k < K; ++k) {
    R *= phi[k - 1];
    pk *= inv_ne;
    const double t = R * pk;
    e.G += t;
    e.Q += k * t;
    q2 += (double)(k * k) * t;
  }
  e.dG = -e.Q * inv_ne;
  e.dQ = -q2 * inv_ne;
  return e;
}

// Step bound of one unknown: x - lam d stays within [x/10, 10 x].
__device__ __forceinline__ double step_bound(double x, double d) {
  if (d > 0.0) return 0.9 * x / d;
  if (d < 0.0) return 9.0 * x / -d;
  return 1.0;
}

// Solves for n_e with the whole wave (blockDim.x == 64).  The neutral
// density of species s and its Saha ratios live in the point's population
// row (pop[s K] and pop[s K + 1 ..]) until the populations overwrite them.
// Returns n_e; *iters receives the step count (negative: no convergence).
__device__ double equilibrium_ne(const Params& P, const Batch& B, int p, double T, double n_tot,
                                 double saha, int* iters) {
  const int S = P.n_species, K = P.n_stages;
  const int lane = threadIdx.x;
  const double kT = kK * T;
  double* row = B.pop + (int64_t)p * S * K;
  const double* A = B.abundance;
  // hydrogen: one ratio
  const double phiH = 2.0 * (kU_HII / kU_HI) * saha * pow(T, 1.5) * exp(-kChiH * kEv / kT);
  // species ratios and the start
  double part = 0.0, asum = 0.0;
  for (int s = lane; s < S; s += 64) {
    double* r = row + s * K;
    for (int k = 0; k + 1 < K; ++k)
      r[1 + k] = 2.0 * (P.part_fn[s * K + k + 1] / P.part_fn[s * K + k]) * saha * pow(T, 1.5) *
                 exp(-P.chi_ev[s * (K - 1) + k] * kEv / kT);
    part += A[s] * (K > 1 ? r[1] : 0.0);
    asum += A[s];
  }
  const double Atot = 1.0 + wave_sum(asum);
  const double nuphi = (phiH + wave_sum(part)) / Atot;
  double ne = fmin(sqrt(n_tot * nuphi), 0.5 * n_tot);
  double nH;
  {
    const double inv = 1.0 / ne;
    nH = (n_tot - ne) / (Atot * elem_gq(&phiH, 2, inv).G);
    for (int s = lane; s < S; s += 64) {
      double* r = row + s * K;
      r[0] = A[s] * (n_tot - ne) / (Atot * elem_gq(r + 1, K, inv).G);
    }
  }
  int it = 0;
  bool done = false;
  while (it < P.ne_max_iter && !done) {
    ++it;
    const double inv = 1.0 / ne;
    const ElemGQ h = elem_gq(&phiH, 2, inv);
    // species sums
    double sNG = 0.0, sNdG = 0.0, sNQ = 0.0, sNdQ = 0.0, sF = 0.0, sC = 0.0, sQAG = 0.0,
           sQC = 0.0, sQF = 0.0;
    for (int s = lane; s < S; s += 64) {
      const double* r = row + s * K;
      const double n = r[0];
      const ElemGQ e = elem_gq(r + 1, K, inv);
      const double fs = n * e.G - A[s] * nH * h.G;
      const double cs = n * e.dG - A[s] * nH * h.dG;
      sNG += n * e.G;
      sNdG += n * e.dG;
      sNQ += n * e.Q;
      sNdQ += n * e.dQ;
      sF += fs;
      sC += cs;
      sQAG += e.Q * A[s] * h.G / e.G;
      sQC += e.Q * cs / e.G;
      sQF += e.Q * fs / e.G;
    }
    sNG = wave_sum(sNG);
    sNdG = wave_sum(sNdG);
    sNQ = wave_sum(sNQ);
    sNdQ = wave_sum(sNdQ);
    sF = wave_sum(sF);
    sC = wave_sum(sC);
    sQAG = wave_sum(sQAG);
    sQC = wave_sum(sQC);
    sQF = wave_sum(sQF);
    // residuals and the reduced 2x2 system in (d_H, d_e)
    const double f0 = nH * h.G + sNG + ne - n_tot;
    const double fe = nH * h.Q + sNQ - ne;
    const double a11 = h.G * Atot;
    const double a12 = (nH * h.dG + sNdG + 1.0) - sC;
    const double b1 = f0 - sF;
    const double a21 = h.Q + sQAG;
    const double a22 = (nH * h.dQ + sNdQ - 1.0) - sQC;
    const double b2 = fe - sQF;
    const double det = a11 * a22 - a12 * a21;
    const double dH = (b1 * a22 - a12 * b2) / det;
    const double de = (a11 * b2 - a21 * b1) / det;
    // step bound over every unknown
    double lam = fmin(1.0, fmin(step_bound(nH, dH), step_bound(ne, de)));
    for (int s = lane; s < S; s += 64) {
      const double* r = row + s * K;
      const double n = r[0];
      const ElemGQ e = elem_gq(r + 1, K, inv);
      const double fs = n * e.G - A[s] * nH * h.G;
      const double cs = n * e.dG - A[s] * nH * h.dG;
      const double ds = (fs + A[s] * h.G * dH - cs * de) / e.G;
      lam = fmin(lam, step_bound(n, ds));
    }
    lam = wave_min(lam);
    // update and the largest relative change
    double rel = 0.0;
    for (int s = lane; s < S; s += 64) {
      double* r = row + s * K;
      const double n = r[0];
      const ElemGQ e = elem_gq(r + 1, K, inv);
      const double fs = n * e.G - A[s] * nH * h.G;
      const double cs = n * e.dG - A[s] * nH * h.dG;
      const double ds = (fs + A[s] * h.G * dH - cs * de) / e.G;
      const double nn = n - lam * ds;
      rel = fmax(rel, fabs(lam * ds) / nn);
      r[0] = nn;
    }
    const double nH1 = nH - lam * dH, ne1 = ne - lam * de;
    rel = fmax(rel, fmax(fabs(lam * dH) / nH1, fabs(lam * de) / ne1));
    rel = wave_max(rel);
    nH = nH1;
    ne = ne1;
    done = rel < kNeTol;
  }
  *iters = done ? it : -it;
  return ne;
}

// One workgroup (one wave) per point: gas state, Saha stage fractions (log
// space), populations N_k/(U_k rho) and the thermal-plus-turbulent
// b = dnu_D/nu0.
__global__ void k_point_state(Params P, Batch B) {
  const int p = blockIdx.x;
  const double T = B.T[p];
  const double Pg = exp10(B.log10P[p]);
  const double kT = kK * T;
  const double saha = pow(2.0 * kPi * kMe * kK / (kH * kH), 1.5);
  double n_e, n_heavy;
  int iters = 0;
  if (P.electrons == 1) {
    n_e = equilibrium_ne(P, B, p, T, Pg / kT, saha, &iters);
    n_heavy = Pg / kT - n_e;
  } else {
    const double pe = P.pe_over_p * Pg;
    n_e = pe / kT;
    n_heavy = (Pg - pe) / kT;
  }
  const int S = P.n_species, K = P.n_stages;
  // sums over species in a fixed order (thread-independent, deterministic)
  double sumA = 0.0, sumAM = 0.0;
  for (int s = 0; s < S; ++s) {
    sumA += B.abundance[s];
    sumAM += B.abundance[s] * P.mass_amu[s];
  }
  const double n_H = n_heavy / (1.0 + sumA);
  const double rho = n_H * kAmu * (kMassH + sumAM);
  if (threadIdx.x == 0) {
    const double t4 = T / 1.0e4;
    PointState ps;
    ps.T = T;
    ps.cS = n_e * pow(t4, 1.0 / 6.0);
    ps.cW = n_heavy * pow(t4, 0.3);
    ps.n_e = n_e;
    ps.n_heavy = n_heavy;
    ps.n_H = n_H;
    ps.rho = rho;
    ps.pad = 0.0;
    B.state[p] = ps;
    B.hmax[p] = 0;
    B.hmax_w[p] = 0;
    B.nsamp[p] = 0ull;
    B.nit[p] = iters;
  }
  const double vt = B.vt_kms[p] * 1e5;
  for (int s = threadIdx.x; s < S; s += blockDim.x) {
    double logf[8];
    logf[0] = 0.0;
    double mx = 0.0;
    for (int k = 0; k + 1 < K; ++k) {
      const double ln_r = log(2.0) + log(P.part_fn[s * K + k + 1]) - log(P.part_fn[s * K + k]) +
                          log(saha) + 1.5 * log(T) - P.chi_ev[s * (K - 1) + k] * kEv / kT -
                          log(n_e);
      logf[k + 1] = logf[k] + ln_r;
      mx = fmax(mx, logf[k + 1]);
    }
    double z = 0.0;
    for (int k = 0; k < K; ++k) z += exp(logf[k] - mx);
    const double lse = mx + log(z);
    for (int k = 0; k < K; ++k) {
      const double f = exp(logf[k] - lse);
      B.pop[(int64_t)p * S * K + s * K + k] =
          B.abundance[s] * n_H * f / (P.part_fn[s * K + k] * rho);
    }
    const double m = P.mass_amu[s] * kAmu;
    const double bb = sqrt(2.0 * kT / m + vt * vt) / kC;
    B.bT[((int64_t)p * S + s) * 2] = bb;              // b = dnu_D / nu_0
    B.bT[((int64_t)p * S + s) * 2 + 1] = 1.0 / bb;    // and 1 / b, so lines multiply
  }
}

hipError_t launch_point_state(hipStream_t st, const Params& P, const Batch& B) {
  if (B.n_points == 0) return hipSuccess;
  hipLaunchKernelGGL(k_point_state, dim3(B.n_points), dim3(64), 0, st, P, B);
  return hipGetLastError();
}

// Per-line constants, loaded once and reused for every point of a batch.
struct LineData {
  double j0s, amp, e_k, hc_k, g_rad, g_stark, g_vdw, thr;
  double ithr, inv_lnq;   // 1/thr and 1/ln q, set by the selection for its window
  int32_t sp, ss;
};

__device__ __forceinline__ LineData load_line(const DevLines& L, int64_t i) {
  LineData d;
  d.j0s = L.j0s[i];
  d.amp = L.amp[i];
  d.e_k = L.e_k[i];
  d.hc_k = L.hc_k[i];
  d.g_rad = L.g_rad[i];
  d.g_stark = L.g_stark[i];
  d.g_vdw = L.g_vdw[i];
  d.thr = L.thr[i];
  d.sp = L.sp[i];
  d.ss = L.ss[i];
  return d;
}

// Factors of a line that depend on T only (shared by the pressures of a T).
struct TFactors {
  double T = -1.0;
  double stim = 0.0, boltz = 0.0;
  __device__ __forceinline__ void update(const LineData& d, double t) {
    if (t == T) return;
    T = t;
    stim = -expm1(-d.hc_k / t);
    boltz = exp(-d.e_k / t);
  }
};

struct LineEval {
  double S, a, b, ib;   // ib = 1 / b
  int32_t jlo, jhi;
  bool surv;
};

// The keep test S H(0, a) >= thr with H(0, a) = erfcx(a), decided where
// possible by the classical bounds of erfcx for a >= 0,
//   2 / (sqrt(pi) (a + sqrt(a^2 + 2))) < erfcx(a) <= 2 / (sqrt(pi) (a + sqrt(a^2 + 4/pi))),
// (Abramowitz and Stegun 7.1.13), each with a margin of 1e-13 for its own
// rounding.  Only lines with thr / U(a) <= S < thr / L(a), a band of at most
// a factor sqrt(pi/2) = 1.25 in S (at a = 0; it narrows as
// 1 + (1 - 2/pi) / (2 a^2) for large a), need erfcx itself, so every
// decision is the one erfcx gives.
__device__ __forceinline__ bool keep_line(double S, double a, double thr) {
  if (!(S >= thr)) return false;                  // erfcx(a) <= 1
  const double lo = 2.0 / (kSqrtPi * (a + sqrt(fma(a, a, 2.0))));
  if (S * lo >= thr * (1.0 + 1e-13)) return true;
  const double hi = 2.0 / (kSqrtPi * (a + sqrt(fma(a, a, 4.0 / kPi))));
  if (S * hi < thr * (1.0 - 1e-13)) return false;
  return S * erfcx(a) >= thr;
}

// The keep test in FP32 first: r = S / thr and a rounded to FP32 (within 1
// ulp each), and the erfcx bounds above compared in FP32 as products,
// 2 r >= (1 + 1e-5) sqrt(pi) (a + sqrt(a^2 + 2)) to keep and
// 2 r < (1 - 1e-5) sqrt(pi) (a + sqrt(a^2 + 4/pi)) to drop (within about
// 6 ulp, 4e-7, with the hardware square root's 1 ulp): they decide every
// line whose r erfcx(a) is more than 1e-5 away from 1 the same way as the
// FP64 test.  1: keep, 0: drop, -1: too close, take the FP64 test.
__device__ __forceinline__ int keep_line32(float rf, float af) {
  constexpr float kSqrtPiF = 1.77245385f;
  if (!(rf < 1e30f) || !(af < 1e15f)) return -1;   // outside the FP32 ranges assumed below
  const float r2 = 2.0f * rf;
  if (r2 >= ((1.0f + 1e-5f) * kSqrtPiF) * (af + __builtin_amdgcn_sqrtf(fmaf(af, af, 2.0f)))) return 1;
  if (r2 < ((1.0f - 1e-5f) * kSqrtPiF) * (af + __builtin_amdgcn_sqrtf(fmaf(af, af, (float)(4.0 / kPi)))))
    return 0;
  return -1;
}

// The library's ln(1 + v) and ln(1 - v), out of line: the window below
// needs them only for |v| > 1/16, which only the strongest hydrogen lines
// reach, above about 100 000 K, and inlined they would hold registers that
// the common path needs.
__device__ __attribute__((noinline)) double2 log1p_pair_lib(double v) {
  return make_double2(log1p(v), log1p(-v));
}

// ln(1 + v) and ln(1 - v) for the window's v = x_w b (x_w <= 500 Doppler
// widths; b is below 1e-4 for every species up to 50 000 K and reaches about
// 1.9e-4 for hydrogen at 200 000 K): from the odd and even parts of the series
// of ln(1 + v), truncated after v^13 and v^12 (the next terms are below
// 1e-18 of the sum for |v| <= 1/16), within 2 ulp of log1p; the library
// log1p beyond.
__device__ __forceinline__ void log1p_pm(double v, double& lp, double& lm) {
  if (fabs(v) <= 0.0625) {
    const double w = v * v;
    double o = 1.0 / 13.0;
    o = fma(o, w, 1.0 / 11.0);
    o = fma(o, w, 1.0 / 9.0);
    o = fma(o, w, 1.0 / 7.0);
    o = fma(o, w, 1.0 / 5.0);
    o = fma(o, w, 1.0 / 3.0);
    o = fma(o, w, 1.0);
    o *= v;
    double e = 1.0 / 12.0;
    e = fma(e, w, 1.0 / 10.0);
    e = fma(e, w, 1.0 / 8.0);
    e = fma(e, w, 1.0 / 6.0);
    e = fma(e, w, 1.0 / 4.0);
    e = fma(e, w, 1.0 / 2.0);
    e = -e * w;
    lp = e + o;
    lm = e - o;
  } else {
    const double2 l = log1p_pair_lib(v);
    lp = l.x;
    lm = l.y;
  }
}

// The FP64 keep test out of line: it is taken only where the FP32 test
// above leaves the decision open, and inlined it would hold registers that
// the common path needs.
__device__ __attribute__((noinline)) bool keep_line64(double S, double a, double thr) {
  return keep_line(S, a, thr);
}

// Strength, damping, selection and window of one line at one point.  The
// keep test is skipped when the caller already knows the line is kept
// (kKept); kWindow false leaves the window out (the emission reads the one
// the selection stored).  bT holds (b, 1/b) per species of the point.
template <bool kKept = false, bool kWindow = true>
__device__ __forceinline__ LineEval eval_line(const Params& P, const LineData& d,
                                              const PointState& ps, const TFactors& tf,
                                              const double* __restrict__ pop,
                                              const double* __restrict__ bT) {
  LineEval e;
  const double b = bT[2 * d.sp], ib = bT[2 * d.sp + 1];
  const double S = d.amp * pop[d.ss] * tf.boltz * tf.stim * ib;
  const double thr = d.thr;
  e.S = S;
  e.b = b;
  e.ib = ib;
  e.a = 0.0;
  e.surv = false;
  e.jlo = 0;
  e.jhi = -1;
  if (!kKept && !(S >= thr)) return e;
  const double a = (d.g_rad + d.g_stark * ps.cS + d.g_vdw * ps.cW) * ib;
  e.a = a;
  if (!kWindow) {
    if (!kKept && !keep_line(S, a, thr)) return e;
    e.surv = true;
    return e;
  }
  if (!kKept) {
    const int k32 = keep_line32((float)(S * d.ithr), (float)a);
    if (k32 == 0 || (k32 < 0 && !keep_line64(S, a, thr))) return e;
  }
  // the window's quotients as products (1/thr once per line and batch, 1/ln q
  // once per thread): a few ulp from the quotients, which can move an edge
  // only where its real value sits on an integer, where either is valid
  // x_w = min(cap, max(x_G, x_L)) with x_G = sqrt(max(0, ln 2r)) and
  // x_L = sqrt(2 r a / sqrt(pi)): one square root of the larger radicand
  // (sqrt is correctly rounded, so monotone, and gives the same value; the
  // Lorentz radicand is never negative, so it also stands for the 0)
  const double r = S * d.ithr;
  const double xw = fmin(P.cap, sqrt(fmax(log(2.0 * r), (2.0 / kSqrtPi) * r * a)));
  double lp, lm;
  log1p_pm(xw * b, lp, lm);
  const double lo = ceil(d.j0s - lp * d.inv_lnq);
  const double hi = floor(d.j0s - lm * d.inv_lnq);
  const double jl = fmax(lo, 0.0);
  const double jh = fmin(hi, (double)(P.N - 1));
  if (jl > jh) return e;
  e.jlo = (int32_t)jl;
  e.jhi = (int32_t)jh;
  e.surv = true;
  return e;
}

constexpr int kWavesK1 = kLineBlock / 64;

// Selection: one thread per line, looping over the batch's points so the
// line's constants are read once per batch.  Writes each line's keep masks
// over the batch's points (kept; kept in the wide class, half-window above
// kNarrowHalf) with one store per line, the
// per-(point, class, block) survivor counts, and per point each class's
// largest half-window and the number of Voigt samples.
__global__ __launch_bounds__(kLineBlock) void k_select(Params P, DevLines L, Batch B) {
  __shared__ int32_t wc[2][kMaxBatch][kWavesK1];
  __shared__ int32_t wh[2][kMaxBatch][kWavesK1];
  __shared__ unsigned long long wn[kMaxBatch][kWavesK1];
  const int64_t i = (int64_t)blockIdx.x * kLineBlock + threadIdx.x;
  const int64_t nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool valid = i < L.n;
  LineData d{};
  if (valid) {
    d = load_line(L, i);
    d.ithr = 1.0 / d.thr;
    d.inv_lnq = 1.0 / P.lnq;
  }
  const int32_t J = (int32_t)rint(d.j0s);
  TFactors tf;
  const int np = B.n_points;
  unsigned long long kept = 0, kwide = 0;
  // the point state through the constant address space (scalar loads; the
  // kernel does not write it)
  typedef const __attribute__((address_space(4))) PointState cps;
  const cps* state = (const cps*)B.state;
  for (int p = 0; p < np; ++p) {
    PointState ps{};   // the fields the line's strength and damping use
    ps.T = state[p].T;
    ps.cS = state[p].cS;
    ps.cW = state[p].cW;
    bool s = false, nar = false;
    int32_t half = 0;
    unsigned long long ns = 0;
    if (valid) {
      tf.update(d, ps.T);
      const LineEval e = eval_line(P, d, ps, tf, B.pop + (int64_t)p * P.n_species * P.n_stages,
                                   B.bT + (int64_t)p * 2 * P.n_species);
      s = e.surv;
      if (s) {
        half = max(J - e.jlo, e.jhi - J) + 1;
        ns = (unsigned long long)(e.jhi - e.jlo + 1);
        nar = half <= kNarrowHalf;
        B.wline[(int64_t)p * B.rec_stride + i] = make_int2(e.jlo, e.jhi);
        kept |= 1ull << p;
        if (!nar) kwide |= 1ull << p;
      }
    }
    const unsigned long long mn = __ballot(s && nar), mw = __ballot(s && !nar);
    int32_t hn = nar ? half : 0, hw = (s && !nar) ? half : 0;
    if (mn | mw) {
      for (int o = 32; o > 0; o >>= 1) {
        hn = max(hn, __shfl_xor(hn, o, 64));
        hw = max(hw, __shfl_xor(hw, o, 64));
        ns += __shfl_xor(ns, o, 64);
      }
    }
    if (lane == 0) {
      wc[0][p][wid] = __popcll(mn);
      wc[1][p][wid] = __popcll(mw);
      wh[0][p][wid] = hn;
      wh[1][p][wid] = hw;
      wn[p][wid] = ns;
    }
  }
  if (valid) B.keep[i] = make_ulonglong2(kept, kwide);
  __syncthreads();
  for (int p = threadIdx.x; p < np; p += blockDim.x) {
    int32_t cn = 0, cw = 0, hn = 0, hw = 0;
    unsigned long long n = 0;
    for (int w = 0; w < kWavesK1; ++w) {
      cn += wc[0][p][w];
      cw += wc[1][p][w];
      hn = max(hn, wh[0][p][w]);
      hw = max(hw, wh[1][p][w]);
      n += wn[p][w];
    }
    B.blk[((int64_t)p * 2 + 0) * nblk + blockIdx.x] = cn;
    B.blk[((int64_t)p * 2 + 1) * nblk + blockIdx.x] = cw;
    if (n) {
      if (hn) atomicMax(B.hmax + p, hn);
      if (hw) atomicMax(B.hmax_w + p, hw);
      atomicAdd(B.nsamp + p, n);
    }
  }
}

hipError_t launch_select(hipStream_t st, const Params& P, const DevLines& L, const Batch& B) {
  if (B.n_points == 0 || L.n == 0) return hipSuccess;
  if (B.n_points > kMaxBatch) return hipErrorInvalidValue;
  const int64_t nblk = n_line_blocks(L.n);
  hipLaunchKernelGGL(k_select, dim3((unsigned)nblk), dim3(kLineBlock), 0, st, P, L, B);
  return hipGetLastError();
}

// Exclusive scan of the per-block survivor counts of one point, each class
// on its own (one workgroup of 1024 threads per point, fixed order:
// deterministic); the narrow class's total places the wide records after it.
__global__ __launch_bounds__(1024) void k_scan(Batch B, int64_t nblk) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry;
  const int p = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int32_t total[2] = {0, 0};
  for (int cls = 0; cls < 2; ++cls) {
    int32_t* c = B.blk + ((int64_t)p * 2 + cls) * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nblk; base += 1024) {
      const int64_t i = base + threadIdx.x;
      const int32_t v = (i < nblk) ? c[i] : 0;
      int32_t x = v;
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
      }
      if (lane == 63) wsum[wid] = x;
      __syncthreads();
      if (threadIdx.x == 0) {
        int32_t run = 0;
        for (int w = 0; w < 16; ++w) {
          const int32_t t = wsum[w];
          wsum[w] = run;
          run += t;
        }
      }
      __syncthreads();
      const int32_t excl = carry + wsum[wid] + x - v;
      if (i < nblk) c[i] = excl;
      __syncthreads();
      if (threadIdx.x == 1023) carry = excl + v;
      __syncthreads();
    }
    total[cls] = carry;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    B.nsurv[p] = total[0] + total[1];
    B.nsurv_n[p] = total[0];
  }
}

hipError_t launch_scan(hipStream_t st, const Params& P, const DevLines& L, const Batch& B) {
  (void)P;
  if (B.n_points == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(B.n_points), dim3(1024), 0, st, B, n_line_blocks(L.n));
  return hipGetLastError();
}

// Survivor emission: the intra-block prefix of the keep masks gives each
// kept line its slot after the block's offset, so the survivor list keeps
// the wavelength order (stable compaction, no atomics on positions).  One
// thread per line and chunk of kEmitChunk points (the grid's y), looping over
// the chunk's points: the offsets are per point and block of lines, so the
// chunks are independent, and short loops keep more loads in flight than one
// loop over the batch (each point waits for its loads).  The per-point values
// every lane shares (the block's offsets, the narrow count, the point state)
// are read through the constant address space: nothing in this kernel writes
// them, and uniform constant loads are scalar loads, issued together with
// one wait (through a generic pointer the record stores make the compiler
// use a vector load and a wait for each).
constexpr int kEmitChunk = 8;

template <bool kRec64>
__global__ __launch_bounds__(kLineBlock) void k_emit(Params P, DevLines L, Batch B) {
  __shared__ int32_t wc[2][kEmitChunk][kWavesK1];
  const int64_t i = (int64_t)blockIdx.x * kLineBlock + threadIdx.x;
  const int64_t nblk = gridDim.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const bool valid = i < L.n;
  const int p0 = (int)blockIdx.y * kEmitChunk;
  const int np = min(B.n_points - p0, kEmitChunk);
  const double inv_lnq = 1.0 / P.lnq;
  const ulonglong2 km = valid ? B.keep[i] : make_ulonglong2(0ull, 0ull);
  // bit p: this line survives at point p0 + p of the batch; wide: ... in the wide class
  const unsigned long long cm = (1ull << np) - 1ull;
  const unsigned long long mine = (km.x >> p0) & cm;
  const unsigned long long wide = (km.y >> p0) & cm;
  for (int p = 0; p < np; ++p) {
    const bool f = (mine >> p) & 1ull, w = (wide >> p) & 1ull;
    const unsigned long long mn = __ballot(f && !w), mw = __ballot(w);
    if (lane == 0) {
      wc[0][p][wid] = __popcll(mn);
      wc[1][p][wid] = __popcll(mw);
    }
  }
  __syncthreads();
  if (!__ballot(mine != 0ull)) return;
  typedef const __attribute__((address_space(4))) int32_t ci32;
  typedef const __attribute__((address_space(4))) PointState cps;
  const ci32* blk = (const ci32*)B.blk;
  const ci32* nsn = (const ci32*)B.nsurv_n;
  const cps* state = (const cps*)B.state;
  LineData d{};
  if (valid) d = load_line(L, i);
  TFactors tf;
  const unsigned long long below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int pc = 0; pc < np; ++pc) {
    const bool f = (mine >> pc) & 1ull;
    const int cls = (int)((wide >> pc) & 1ull);
    const unsigned long long mn = __ballot(f && cls == 0), mw = __ballot(f && cls == 1);
    if (!(mn | mw)) continue;
    const int p = p0 + pc;   // the point in the batch
    const int32_t off_n = blk[((int64_t)p * 2 + 0) * nblk + blockIdx.x];
    const int32_t off_w = blk[((int64_t)p * 2 + 1) * nblk + blockIdx.x] + nsn[p];
    PointState ps{};   // the fields the line's strength and damping use
    ps.T = state[p].T;
    ps.cS = state[p].cS;
    ps.cW = state[p].cW;
    if (!f) continue;
    int32_t off = cls ? off_w : off_n;
    for (int w = 0; w < wid; ++w) off += wc[cls][pc][w];
    off += __popcll((cls ? mw : mn) & below);
    tf.update(d, ps.T);
    LineEval e = eval_line<true, false>(P, d, ps, tf, B.pop + (int64_t)p * P.n_species * P.n_stages,
                                        B.bT + (int64_t)p * 2 * P.n_species);
    const int2 wl = B.wline[(int64_t)p * B.rec_stride + i];
    e.jlo = wl.x;
    e.jhi = wl.y;
    const double Jd = rint(d.j0s);
    const int32_t J = (int32_t)Jd;
    const int64_t slot = (int64_t)p * B.rec_stride + off;
    B.win[slot] = make_int2(e.jlo, e.jhi);
    // c1 = ln q / b; the zone half-widths ceil(1.02 R / c1) + 2 as
    // products (1 / ln q once per thread): a few ulp from the quotients,
    // which can move a half-width only at an exact tie, where both are valid
    const double c1 = P.lnq * e.ib;
    const double b_lnq = e.b * inv_lnq;
    int32_t czh, z40 = -1;
    if (kRec64) {
      czh = e.a < kFarR64 ? zone_half_b(kFarR64, b_lnq) : -1;
      z40 = e.a < kFar4R64 ? zone_half_b(kFar4R64, b_lnq) : -1;
      B.wz[slot] = make_int2(J, z40);
    } else {
      // no zone: -32768, which the Voigt kernel's row masks read as empty
      const int32_t far = e.a < kFarR32 ? min(zone_half_b(kFarR32, b_lnq), 32767) : -32768;
      const int32_t ring = e.a < kRingR32 ? min(zone_half_b(kRingR32, b_lnq), 32767) : -32768;
      czh = (int32_t)(((uint32_t)ring << 16) | ((uint32_t)far & 0xffffu));
      B.wz[slot] = make_int2(J, czh);
    }
    if (kRec64) {
      Rec64 r;
      r.J = J;
      r.jlo = e.jlo;
      r.jhi = e.jhi;
      r.czh = czh;
      r.z40 = z40;
      r.li = (int32_t)i;
      r.pad0 = r.pad1 = 0;
      r.phi = d.j0s - Jd;
      r.S = e.S;
      r.y = e.a;
      r.c1 = c1;
      reinterpret_cast<Rec64*>(B.rec)[slot] = r;
    } else {
      Rec32 r;
      r.J = J;
      r.jlo = e.jlo;
      r.jhi = e.jhi;
      r.czh = czh;
      r.phi = (float)(d.j0s - Jd);
      const double C1 = e.S * e.a * (1.0 / kSqrtPi);
      if (e.a >= 1.0e4) {
        // Lorentz limit in u = x / a
        r.c1 = (float)(c1 / e.a);
        r.A = (float)(C1 / (e.a * e.a));
        r.B = 0.0f;
        r.D = 1.0f;
        r.E = 0.0f;
      } else {
        // two-node rule (t^2 = 1/2)
        r.c1 = (float)c1;
        r.A = r.B = (float)C1;
        r.D = (float)(e.a * e.a - 0.5);
        r.E = (float)(2.0 * e.a * e.a);
      }
      r.S = (float)e.S;
      r.y = (float)e.a;
      reinterpret_cast<Rec32*>(B.rec)[slot] = r;
    }
  }
}

hipError_t launch_emit(hipStream_t st, const Params& P, const DevLines& L, const Batch& B,
                       int rec64) {
  if (B.n_points == 0 || L.n == 0) return hipSuccess;
  if (B.n_points > kMaxBatch) return hipErrorInvalidValue;
  const int64_t nblk = n_line_blocks(L.n);
  const dim3 grid((unsigned)nblk, (unsigned)((B.n_points + kEmitChunk - 1) / kEmitChunk));
  if (rec64)
    hipLaunchKernelGGL(k_emit<true>, grid, dim3(kLineBlock), 0, st, P, L, B);
  else
    hipLaunchKernelGGL(k_emit<false>, grid, dim3(kLineBlock), 0, st, P, L, B);
  return hipGetLastError();
}

}  // namespace odf

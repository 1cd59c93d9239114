// Voigt scatter-sum onto the fine grid (gfx950): every kept line adds
// S * H(x_j, a) to the fine-grid opacity inside its window (Sec. 2.1,
// eq. l_nu_line; App. E second stage).  H(x, a) = Re w(x + i a).
//
// Owner-computes tiling: a wave owns 1024 consecutive fine points (16 rows
// of 64 lanes, one point per lane per row) and keeps their sums in
// registers.  It walks the wavelength-sorted survivors whose centres lie
// within the point's largest half-window of its points, tests 64 windows at
// a time with one ballot, and for each intersecting line evaluates only the
// rows the window covers.  No atomics: each point is summed by one lane in
// the survivors' wavelength order, so results are bit-reproducible.
//
// Re w is evaluated in real arithmetic only, so that its relative accuracy
// holds where Re w << |w| (far wings of weakly damped lines):
//  - far from the core, a Gauss-Hermite quadrature of
//    H = (a/pi) int exp(-t^2) / ((x - t)^2 + a^2) dt, written as one fraction
//    of positive terms (nodes and weights computed at plan time);
//  - near the core, the trapezoidal rule for the same integral with the
//    contribution of the integrand's pole at t = x + i a added in closed
//    form (the error of the corrected rule is of order exp(-pi^2/h^2)); the
//    node grid is shifted by half a step when x lies near a node.
// Mixed precision uses FP32 with Kahan-compensated sums (every summand is
// positive, so the compensated error bound is relative to the sum); the
// plain path uses FP64 throughout.
#include "odf_internal.h"

namespace odf {

namespace {

constexpr float kInvSqrtPiF = 0.56418958354775628695f;
constexpr float kPiF = 3.14159265358979323846f;

__device__ __forceinline__ int xcd_remap(int bid, int total) {
  // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a
  // contiguous range of (point, tile) so neighbouring tiles, which read the
  // same survivors, share that XCD's L2.
  const int per = (total + 7) / 8;
  return (bid & 7) * per + (bid >> 3);
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
  const float yv = v - c;
  const float t = s + yv;
  c = (t - s) - yv;
  s = t;
}

template <typename Rec>
__device__ __forceinline__ int lower_bound_J(const Rec* __restrict__ r, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (r[mid].J < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <typename Rec>
__device__ __forceinline__ int upper_bound_J(const Rec* __restrict__ r, int n, int key) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (r[mid].J <= key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------- FP32 ----

// General FP32 H(x, y) for any |z| (core rows).
__device__ __forceinline__ float voigt32(float x, float y, const QuadConsts& Q) {
  const float x2 = x * x, y2 = y * y, r2 = x2 + y2;
  if (r2 >= kFarR32 * kFarR32) {
    const float u = r2 + Q.gh2_t2;
    return (y * kInvSqrtPiF) * u * __builtin_amdgcn_rcpf(fmaf(u, u, -4.0f * Q.gh2_t2 * x2));
  }
  if (r2 >= kRingR32 * kRingR32) {
    const float p1 = r2 + Q.gh4_t2[0], p2 = r2 + Q.gh4_t2[1];
    const float d1 = fmaf(p1, p1, -4.0f * Q.gh4_t2[0] * x2);
    const float d2 = fmaf(p2, p2, -4.0f * Q.gh4_t2[1] * x2);
    const float num = fmaf(Q.gh4_w[0] * p1, d2, Q.gh4_w[1] * p2 * d1);
    return 2.0f * y * num * __builtin_amdgcn_rcpf(d1 * d2);
  }
  // pole-corrected trapezoid, nodes t_k = (k + delta) h
  const float invh = 1.0f / kTrap32H;
  const float hx = x * invh;
  const float fr = hx - rintf(hx);
  const bool sh = fabsf(fr) < 0.25f;
  const float delta = sh ? 0.5f : 0.0f;
  float num = 0.0f, den = 1.0f;
#pragma unroll
  for (int k = -kTrap32Half; k <= kTrap32Half; ++k) {
    const float t = ((float)k + delta) * kTrap32H;
    const float dd = x - t;
    const float D = fmaf(dd, dd, y2);
    const float ck = sh ? Q.tr32_ch[k + kTrap32Half] : Q.tr32_ci[k + kTrap32Half];
    num = fmaf(num, D, ck * den);
    den *= D;
  }
  float h = y * num / den;
  if (y < kPiF * invh) {
    // Re[ 2 e^{-z^2} / (1 -/+ e^{-2 pi i z / h}) ] with E = e^{-2 pi y/h} e^{2 pi i x/h}
    const float e2 = 2.0f * kPiF * y * invh;
    const float mag = __expf(y2 - x2 - e2);
    const float ep = __expf(-e2);
    float sph, cph, sth, cth;
    sincospif(2.0f * hx, &sph, &cph);
    sincospif(2.0f * hx - 2.0f * x * y / kPiF, &sth, &cth);
    const float sgn = sh ? 1.0f : -1.0f;
    const float dre = fmaf(ep, cph, sgn), dim = ep * sph;
    h += 2.0f * mag * (cth * dre + sth * dim) / fmaf(dre, dre, dim * dim);
  }
  return h;
}

template <bool kLorentz>
__device__ __forceinline__ void far_rows32(const Rec32& r, int t_lo, int lane, int r_lo, int r_hi,
                                           int rc_lo, int rc_hi, float c1, float c2, float c3,
                                           float C1, float C2, float (&as)[kRows],
                                           float (&ac)[kRows]) {
  const int ib = r.J - t_lo - lane;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    if (rr < r_lo || rr > r_hi) continue;
    if (rr >= rc_lo && rr <= rc_hi) continue;
    const float d = (float)(ib - 64 * rr) + r.phi;
    const float x = d * fmaf(d, fmaf(d, c3, c2), c1);
    const float x2 = x * x;
    float v;
    if (kLorentz) {
      v = C1 * __builtin_amdgcn_rcpf(x2 + C2);
    } else {
      const float u = x2 + C2;
      v = (u * C1) * __builtin_amdgcn_rcpf(fmaf(u, u, -2.0f * x2));
    }
    const int rs = t_lo + 64 * rr;
    if (!(rs >= r.jlo && rs + 63 <= r.jhi)) {
      const int j = rs + lane;
      v = (j >= r.jlo && j <= r.jhi) ? v : 0.0f;
    }
    kahan_add(as[rr], ac[rr], v);
  }
}

__device__ __forceinline__ void line32(const Rec32& r, int t_lo, int t_hi, int lane, float lnq,
                                       const QuadConsts& Q, float (&as)[kRows], float (&ac)[kRows],
                                       float* __restrict__ ls, float* __restrict__ lc) {
  const int jl = max(r.jlo, t_lo) - t_lo;
  const int jh = min(r.jhi, t_hi) - t_lo;
  const int r_lo = jl >> 6, r_hi = jh >> 6;
  // x = expm1(d ln q) / b = d (c1 + c2 d + c3 d^2) + O(d^4 ln q^3), |d ln q| <= 0.031
  const float c1 = r.c1;
  const float c2 = c1 * lnq * 0.5f;
  const float c3 = c1 * lnq * lnq * (1.0f / 6.0f);
  const float y = r.y;
  // rows that may contain |z| < 15 need the general evaluation
  int rc_lo = 1, rc_hi = 0;
  if (y < kFarR32) {
    const float Dc = kFarR32 * 1.02f / c1 + 2.0f;
    const float ctr = (float)(r.J - t_lo) + r.phi;
    rc_lo = ((int)floorf(ctr - Dc)) >> 6;
    rc_hi = ((int)ceilf(ctr + Dc)) >> 6;
  }
  if (y >= 1.0e4f) {
    // Lorentz limit: the Gauss-Hermite pair correction is below 1/(2 y^2)
    far_rows32<true>(r, t_lo, lane, r_lo, r_hi, rc_lo, rc_hi, c1, c2, c3,
                     r.S * y * kInvSqrtPiF, y * y, as, ac);
  } else {
    far_rows32<false>(r, t_lo, lane, r_lo, r_hi, rc_lo, rc_hi, c1, c2, c3,
                      r.S * y * kInvSqrtPiF, fmaf(y, y, Q.gh2_t2), as, ac);
  }
  const int g_lo = max(r_lo, rc_lo), g_hi = min(r_hi, rc_hi);
  const int ib = r.J - t_lo - lane;
  for (int rr = g_lo; rr <= g_hi; ++rr) {
    const float d = (float)(ib - 64 * rr) + r.phi;
    const float x = d * fmaf(d, fmaf(d, c3, c2), c1);
    float v = r.S * voigt32(x, y, Q);
    const int j = t_lo + 64 * rr + lane;
    v = (j >= r.jlo && j <= r.jhi) ? v : 0.0f;
    const int o = rr * 64 + lane;
    float s = ls[o], c = lc[o];
    kahan_add(s, c, v);
    ls[o] = s;
    lc[o] = c;
  }
}

__global__ __launch_bounds__(256) void k_voigt32(Params P, Batch B, QuadConsts Q,
                                                 int tiles_per_point, int total) {
  __shared__ float lds_s[kWavesPerWG][kWavePoints];
  __shared__ float lds_c[kWavesPerWG][kWavePoints];
  const int logical = xcd_remap(blockIdx.x, total);
  if (logical >= total) return;
  const int p = logical / tiles_per_point;
  const int tile = logical - p * tiles_per_point;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int N = (int)P.N;
  const int t_lo = tile * kWGPoints + wid * kWavePoints;
  if (t_lo >= N) return;
  const int t_hi = min(t_lo + kWavePoints - 1, N - 1);
  float* ls = lds_s[wid];
  float* lc = lds_c[wid];
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    ls[rr * 64 + lane] = 0.0f;
    lc[rr * 64 + lane] = 0.0f;
  }
  float as[kRows], ac[kRows];
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    as[rr] = 0.0f;
    ac[rr] = 0.0f;
  }
  const Rec32* __restrict__ rec = reinterpret_cast<const Rec32*>(B.rec) + p * B.rec_stride;
  const int2* __restrict__ win = B.win + p * B.rec_stride;
  const int ns = B.nsurv[p];
  const int H = B.hmax[p];
  const float lnq = (float)P.lnq;
  const int c0 = lower_bound_J(rec, ns, t_lo - H);
  const int c1 = upper_bound_J(rec, ns, t_hi + H);
  for (int base = c0; base < c1; base += 64) {
    const int i = base + lane;
    int2 w = make_int2(1, 0);
    if (i < c1) w = win[i];
    unsigned long long m = __ballot(w.x <= t_hi && w.y >= t_lo);
    while (m) {
      const int k = __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1);
      m &= m - 1;
      const Rec32 r = rec[base + k];
      line32(r, t_lo, t_hi, lane, lnq, Q, as, ac, ls, lc);
    }
  }
  float* kap = reinterpret_cast<float*>(B.kappa) + p * B.kappa_stride;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    const int j = t_lo + rr * 64 + lane;
    const int o = rr * 64 + lane;
    if (j <= t_hi) kap[j] = (as[rr] - ac[rr]) + (ls[o] - lc[o]);
  }
}

// ---------------------------------------------------------------- FP64 ----

// Eight-node Gauss-Hermite pair sum for |z| >= 10, one division.
__device__ __forceinline__ double gh8(double x2, double y, double r2, const QuadConsts& Q) {
  const double p1 = r2 + Q.gh8_t2[0];
  const double d1 = fma(p1, p1, -4.0 * Q.gh8_t2[0] * x2);
  double num = Q.gh8_w[0] * p1, den = d1;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const double pk = r2 + Q.gh8_t2[k];
    const double dk = fma(pk, pk, -4.0 * Q.gh8_t2[k] * x2);
    num = fma(num, dk, Q.gh8_w[k] * pk * den);
    den *= dk;
  }
  return 2.0 * y * num / den;
}

__device__ __forceinline__ double voigt64(double x, double y, const QuadConsts& Q) {
  const double x2 = x * x, y2 = y * y, r2 = x2 + y2;
  if (r2 >= kFarR64 * kFarR64) return gh8(x2, y, r2, Q);
  const double invh = 1.0 / kTrap64H;
  const double hx = x * invh;
  const double fr = hx - rint(hx);
  const bool sh = fabs(fr) < 0.25;
  const double delta = sh ? 0.5 : 0.0;
  double num = 0.0, den = 1.0;
#pragma unroll
  for (int k = -kTrap64Half; k <= kTrap64Half; ++k) {
    const double t = ((double)k + delta) * kTrap64H;
    const double dd = x - t;
    const double D = fma(dd, dd, y2);
    const double ck = sh ? Q.tr64_ch[k + kTrap64Half] : Q.tr64_ci[k + kTrap64Half];
    num = fma(num, D, ck * den);
    den *= D;
  }
  double h = y * num / den;
  if (y < kPi * invh) {
    const double e2 = 2.0 * kPi * y * invh;
    const double mag = exp(y2 - x2 - e2);
    const double ep = exp(-e2);
    double sph, cph, sth, cth;
    sincospi(2.0 * hx, &sph, &cph);
    sincospi(2.0 * hx - 2.0 * x * y / kPi, &sth, &cth);
    const double sgn = sh ? 1.0 : -1.0;
    const double dre = fma(ep, cph, sgn), dim = ep * sph;
    h += 2.0 * mag * (cth * dre + sth * dim) / fma(dre, dre, dim * dim);
  }
  return h;
}

// x = expm1(u)/b = d c1 E(u), u = d ln q, E(u) = expm1(u)/u (Taylor to u^7,
// |u| <= 0.031 so the truncation is below 1e-18 relative).
__device__ __forceinline__ double x_of_d64(double d, double c1, double lnq) {
  const double u = d * lnq;
  double e = 1.0 / 40320.0;
  e = fma(e, u, 1.0 / 5040.0);
  e = fma(e, u, 1.0 / 720.0);
  e = fma(e, u, 1.0 / 120.0);
  e = fma(e, u, 1.0 / 24.0);
  e = fma(e, u, 1.0 / 6.0);
  e = fma(e, u, 0.5);
  e = fma(e, u, 1.0);
  return d * c1 * e;
}

__device__ __forceinline__ void line64(const Rec64& r, int t_lo, int t_hi, int lane, double lnq,
                                       const QuadConsts& Q, double (&as)[kRows],
                                       double* __restrict__ ls) {
  const int jl = max(r.jlo, t_lo) - t_lo;
  const int jh = min(r.jhi, t_hi) - t_lo;
  const int r_lo = jl >> 6, r_hi = jh >> 6;
  const double c1 = r.c1, y = r.y, S = r.S;
  int rc_lo = 1, rc_hi = 0;
  if (y < kFarR64) {
    const double Dc = kFarR64 * 1.02 / c1 + 2.0;
    const double ctr = (double)(r.J - t_lo) + r.phi;
    rc_lo = ((int)floor(ctr - Dc)) >> 6;
    rc_hi = ((int)ceil(ctr + Dc)) >> 6;
  }
  const double y2 = y * y;
  const int ib = r.J - t_lo - lane;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    if (rr < r_lo || rr > r_hi) continue;
    if (rr >= rc_lo && rr <= rc_hi) continue;
    const double d = (double)(ib - 64 * rr) + r.phi;
    const double x = x_of_d64(d, c1, lnq);
    const double x2 = x * x;
    double v = S * gh8(x2, y, x2 + y2, Q);
    const int rs = t_lo + 64 * rr;
    if (!(rs >= r.jlo && rs + 63 <= r.jhi)) {
      const int j = rs + lane;
      v = (j >= r.jlo && j <= r.jhi) ? v : 0.0;
    }
    as[rr] += v;
  }
  const int g_lo = max(r_lo, rc_lo), g_hi = min(r_hi, rc_hi);
  for (int rr = g_lo; rr <= g_hi; ++rr) {
    const double d = (double)(ib - 64 * rr) + r.phi;
    const double x = x_of_d64(d, c1, lnq);
    double v = S * voigt64(x, y, Q);
    const int j = t_lo + 64 * rr + lane;
    v = (j >= r.jlo && j <= r.jhi) ? v : 0.0;
    ls[rr * 64 + lane] += v;
  }
}

__global__ __launch_bounds__(256) void k_voigt64(Params P, Batch B, QuadConsts Q,
                                                 int tiles_per_point, int total) {
  __shared__ double lds_s[kWavesPerWG][kWavePoints];
  const int logical = xcd_remap(blockIdx.x, total);
  if (logical >= total) return;
  const int p = logical / tiles_per_point;
  const int tile = logical - p * tiles_per_point;
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int N = (int)P.N;
  const int t_lo = tile * kWGPoints + wid * kWavePoints;
  if (t_lo >= N) return;
  const int t_hi = min(t_lo + kWavePoints - 1, N - 1);
  double* ls = lds_s[wid];
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) ls[rr * 64 + lane] = 0.0;
  double as[kRows];
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) as[rr] = 0.0;
  const Rec64* __restrict__ rec = reinterpret_cast<const Rec64*>(B.rec) + p * B.rec_stride;
  const int2* __restrict__ win = B.win + p * B.rec_stride;
  const int ns = B.nsurv[p];
  const int H = B.hmax[p];
  const double lnq = P.lnq;
  const int c0 = lower_bound_J(rec, ns, t_lo - H);
  const int c1 = upper_bound_J(rec, ns, t_hi + H);
  for (int base = c0; base < c1; base += 64) {
    const int i = base + lane;
    int2 w = make_int2(1, 0);
    if (i < c1) w = win[i];
    unsigned long long m = __ballot(w.x <= t_hi && w.y >= t_lo);
    while (m) {
      const int k = __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1);
      m &= m - 1;
      const Rec64 r = rec[base + k];
      line64(r, t_lo, t_hi, lane, lnq, Q, as, ls);
    }
  }
  double* kap = reinterpret_cast<double*>(B.kappa) + p * B.kappa_stride;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    const int j = t_lo + rr * 64 + lane;
    if (j <= t_hi) kap[j] = as[rr] + ls[rr * 64 + lane];
  }
}

}  // namespace

hipError_t launch_voigt(hipStream_t st, const Params& P, const Batch& B, const QuadConsts& Q) {
  if (B.n_points == 0) return hipSuccess;
  const int tiles = (int)((P.N + kWGPoints - 1) / kWGPoints);
  const int total = tiles * B.n_points;
  const int grid = ((total + 7) / 8) * 8;
  if (P.precision == 1)
    hipLaunchKernelGGL(k_voigt32, dim3(grid), dim3(256), 0, st, P, B, Q, tiles, total);
  else
    hipLaunchKernelGGL(k_voigt64, dim3(grid), dim3(256), 0, st, P, B, Q, tiles, total);
  return hipGetLastError();
}

}  // namespace odf

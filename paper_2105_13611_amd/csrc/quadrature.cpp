// Quadrature constants for the Voigt kernels, computed at plan time.
//
// Gauss-Hermite rules (weight e^{-t^2}): nodes are the roots of the
// physicists' Hermite polynomial H_n, found by sign-change bracketing and
// bisection in long double; weights are
//   w_k = 2^{n-1} n! sqrt(pi) / (n^2 H_{n-1}(t_k)^2).
// Trapezoidal-rule weights are (h/pi) e^{-t^2} at the nodes t = k h and
// t = (k + 1/2) h, zero beyond the truncation |t| > tmax.  The small-damping
// series table holds cubic pieces of the Dawson-derivative terms.
#include <cmath>
#include <vector>

#include "odf_internal.h"

namespace odf {

namespace {

long double hermite(int n, long double t, long double* prev = nullptr) {
  long double h0 = 1.0L, h1 = 2.0L * t;
  if (n == 0) {
    if (prev) *prev = 0.0L;
    return h0;
  }
  for (int k = 1; k < n; ++k) {
    const long double h2 = 2.0L * t * h1 - 2.0L * k * h0;
    h0 = h1;
    h1 = h2;
  }
  if (prev) *prev = h0;
  return h1;
}

// positive nodes (ascending) and their weights of the n-point rule, n even
void gauss_hermite_positive(int n, std::vector<long double>& t, std::vector<long double>& w) {
  t.clear();
  w.clear();
  const long double tmax = std::sqrt(2.0L * n + 1.0L) + 1.0L;
  const long double step = 1e-4L;
  long double a = step * 0.5L, fa = hermite(n, a);
  for (long double b = a + step; b < tmax; b += step) {
    const long double fb = hermite(n, b);
    if ((fa < 0) != (fb < 0)) {
      long double lo = a, hi = b, flo = fa;
      for (int it = 0; it < 200; ++it) {
        const long double mid = 0.5L * (lo + hi);
        const long double fm = hermite(n, mid);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      t.push_back(0.5L * (lo + hi));
    }
    a = b;
    fa = fb;
  }
  long double fact = 1.0L;
  for (int k = 2; k <= n; ++k) fact *= k;
  const long double sqrt_pi = std::sqrt(3.14159265358979323846264338327950288L);
  for (long double tk : t) {
    const long double hm1 = hermite(n - 1, tk);
    w.push_back(std::pow(2.0L, n - 1) * fact * sqrt_pi / ((long double)n * n * hm1 * hm1));
  }
}

// n-th derivative of Dawson's function F(x) = e^{-x^2} int_0^x e^{t^2} dt,
// from Rybicki's sampling-theorem representation
//   F(x) = lim_{h -> 0} pi^{-1/2} sum_{m odd} e^{-(x - m h)^2} / m
// (G. B. Rybicki, Computers in Physics 3 (1989) 85).  With h = 0.2 the
// representation error is of order e^{-(pi / 2h)^2} ~ 1e-27; each Gaussian is
// differentiated exactly, d^n/dx^n e^{-u^2} = (-1)^n H_n(u) e^{-u^2}.  Unlike
// the derivative recurrence F^(n+1) = -2x F^(n) - 2n F^(n-1), this keeps its
// relative accuracy for x of order 10.
long double dawson_derivative(int n, long double x) {
  const long double h = 0.2L, L = 9.5L;
  const long double inv_sqrt_pi = 0.564189583547756286948079451560772586L;
  const long long m_lo = (long long)std::floor((x - L) / h) - 1;
  const long long m_hi = (long long)std::ceil((x + L) / h) + 1;
  long double sum = 0.0L;
  for (long long m = m_lo; m <= m_hi; ++m) {
    if ((m & 1LL) == 0) continue;
    const long double u = x - (long double)m * h;
    sum += hermite(n, u) * std::exp(-u * u) / (long double)m;
  }
  return ((n & 1) ? -sum : sum) * inv_sqrt_pi;
}

// (-1)^{(n+1)/2} (2/sqrt(pi)) / n!, so that T_n = coefficient * F^(n).
long double series_coefficient(int n) {
  const long double two_over_sqrt_pi = 1.128379167095512573896158903121545172L;
  long double fact = 1.0L;
  for (int k = 2; k <= n; ++k) fact *= k;
  const long double sg = (((n + 1) / 2) & 1) ? -1.0L : 1.0L;
  return sg * two_over_sqrt_pi / fact;
}

// Cubic Hermite pieces of T_n against s = 1/(1 + x^2).  dT/ds = T'(x) dx/ds
// with dx/ds = -(1 + x^2)^2 / (2x); at s = 1 (x = 0, T even) dT/ds =
// -T''(0)/2; at s = 0 (x -> infinity) T_1 ~ s / sqrt(pi) and T_n = O(s^2)
// for n >= 3.
void series_table(QuadConsts& Q) {
  constexpr int NS = kSerIntervals;
  const long double inv_sqrt_pi = 0.564189583547756286948079451560772586L;
  for (int k = 0; k < kSerTerms; ++k) {
    const int n = 2 * k + 1;
    const long double c = series_coefficient(n);
    std::vector<long double> v(NS + 1), d(NS + 1);
    for (int i = 0; i <= NS; ++i) {
      const long double s = (long double)i / NS;
      if (i == 0) {
        v[i] = 0.0L;
        d[i] = (n == 1) ? inv_sqrt_pi : 0.0L;
      } else if (i == NS) {
        v[i] = c * dawson_derivative(n, 0.0L);
        d[i] = -0.5L * c * dawson_derivative(n + 2, 0.0L);
      } else {
        const long double x = std::sqrt(1.0L / s - 1.0L);
        v[i] = c * dawson_derivative(n, x);
        d[i] = c * dawson_derivative(n + 1, x) * (-(1.0L + x * x) * (1.0L + x * x) / (2.0L * x));
      }
    }
    const long double hs = 1.0L / NS;
    for (int i = 0; i < NS; ++i) {
      const long double v0 = v[i], v1 = v[i + 1], d0 = d[i] * hs, d1 = d[i + 1] * hs;
      Q.ser[k][i][0] = (float)v0;
      Q.ser[k][i][1] = (float)d0;
      Q.ser[k][i][2] = (float)(3.0L * (v1 - v0) - 2.0L * d0 - d1);
      Q.ser[k][i][3] = (float)(2.0L * (v0 - v1) + d0 + d1);
    }
  }
}

}  // namespace

QuadConsts make_quad_consts() {
  QuadConsts Q{};
  const long double pi = 3.14159265358979323846264338327950288L;
  std::vector<long double> t, w;
  gauss_hermite_positive(2, t, w);
  Q.gh2_t2 = (float)(t[0] * t[0]);
  gauss_hermite_positive(4, t, w);
  for (int k = 0; k < 2; ++k) {
    Q.gh4_t2[k] = (float)(t[k] * t[k]);
    Q.gh4_w[k] = (float)(w[k] / pi);
    Q.gh4_t2d[k] = (double)(t[k] * t[k]);
    Q.gh4_wd[k] = (double)(w[k] / pi);
  }
  gauss_hermite_positive(8, t, w);
  for (int k = 0; k < 4; ++k) {
    Q.gh8_t2[k] = (double)(t[k] * t[k]);
    Q.gh8_w[k] = (double)(w[k] / pi);
  }
  for (int k = -kTrap32Half; k <= kTrap32Half; ++k) {
    const long double h = kTrap32H, tm = kTrap32Tmax;
    const long double ti = k * h, th = (k + 0.5L) * h;
    Q.tr32_ci[k + kTrap32Half] = std::fabs(ti) <= tm ? (float)(h / pi * std::exp(-ti * ti)) : 0.0f;
    Q.tr32_ch[k + kTrap32Half] = std::fabs(th) <= tm ? (float)(h / pi * std::exp(-th * th)) : 0.0f;
  }
  for (int k = -kTrap64Half; k <= kTrap64Half; ++k) {
    const long double h = kTrap64H, tm = kTrap64Tmax;
    const long double ti = k * h, th = (k + 0.5L) * h;
    Q.tr64_ci[k + kTrap64Half] = std::fabs(ti) <= tm ? (double)(h / pi * std::exp(-ti * ti)) : 0.0;
    Q.tr64_ch[k + kTrap64Half] = std::fabs(th) <= tm ? (double)(h / pi * std::exp(-th * th)) : 0.0;
  }
  for (int n = 0; n < kFFNodes; ++n) {
    const long double th = (2 * n + 1) * pi / (2 * kFFNodes);
    Q.ff_s[n] = (float)std::cos(th);
    Q.ff_w[n] = (float)((n % 2 ? -1.0L : 1.0L) * std::sin(th));
  }
  for (int l = 0; l < 64; ++l) {
    const long double th = (2 * (l % kFFNodes) + 1) * pi / (2 * kFFNodes);
    const long double half = 0.5L * (kFFQuarter - 1);
    Q.ff_off[l] = (float)(kFFQuarter * (l / kFFNodes) + half + half * std::cos(th));
    Q.ff_off64[l] = (double)(kFFQuarter * (l / kFFNodes) + half + half * std::cos(th));
  }
  // whole-tile tiers: Chebyshev points of the first kind over the tile's
  // 1024 points, and the Lagrange basis values at the quarter nodes from the
  // barycentric formula, normalised (no quarter node coincides with a tile
  // node: the closest pair is 0.002 points apart)
  {
    const long double half_t = 0.5L * (kWavePoints - 1);
    const long double half_q = 0.5L * (kFFQuarter - 1);
    int base = 0;
    for (int K = 32; K >= 8; K /= 2) {
      for (int n = 0; n < K; ++n)
        Q.ff_toff[base + n] = (float)(half_t + half_t * std::cos((2 * n + 1) * pi / (2 * K)));
      for (int l = 0; l < 64; ++l) {
        const long double th_q = (2 * (l % kFFNodes) + 1) * pi / (2 * kFFNodes);
        const long double xq = kFFQuarter * (l / kFFNodes) + half_q + half_q * std::cos(th_q);
        const long double t = (xq - half_t) / half_t;
        long double r[32], sum = 0.0L;
        for (int n = 0; n < K; ++n) {
          const long double th = (2 * n + 1) * pi / (2 * K);
          r[n] = (n % 2 ? -1.0L : 1.0L) * std::sin(th) / (t - std::cos(th));
          sum += r[n];
        }
        for (int n = 0; n < K; ++n) Q.ff_V[base + n][l] = (float)(r[n] / sum);
      }
      base += K;
    }
  }
  // barycentric weights w_n / (t - s_n), normalised, at the 256 points of a
  // quarter (t in [-1, 1]; no point coincides with a node)
  for (int k = 0; k < kFFQuarter; ++k) {
    const long double half = 0.5L * (kFFQuarter - 1);
    const long double t = ((long double)k - half) / half;
    long double r[kFFNodes], sum = 0.0L;
    for (int n = 0; n < kFFNodes; ++n) {
      const long double th = (2 * n + 1) * pi / (2 * kFFNodes);
      r[n] = (n % 2 ? -1.0L : 1.0L) * std::sin(th) / (t - std::cos(th));
      sum += r[n];
    }
    for (int n = 0; n < kFFNodes; ++n) Q.ff_M64[k][n] = (double)(r[n] / sum);
  }
  series_table(Q);
  return Q;
}

}  // namespace odf

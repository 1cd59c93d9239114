// Quadrature constants for the Voigt kernels, computed at plan time.
//
// Gauss-Hermite rules (weight e^{-t^2}): nodes are the roots of the
// physicists' Hermite polynomial H_n, found by sign-change bracketing and
// bisection in long double; weights are
//   w_k = 2^{n-1} n! sqrt(pi) / (n^2 H_{n-1}(t_k)^2).
// Trapezoidal-rule weights are (h/pi) e^{-t^2} at the nodes t = k h and
// t = (k + 1/2) h, zero beyond the truncation |t| > tmax.
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
  return Q;
}

}  // namespace odf

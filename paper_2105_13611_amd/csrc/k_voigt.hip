// Voigt scatter-sum onto the fine grid (gfx950): every kept line adds
// S * H(x_j, a) to the fine-grid opacity inside its window (Sec. 2.1,
// eq. l_nu_line; App. E second stage).  H(x, a) = Re w(x + i a).
//
// Owner-computes tiling: a wave owns 1024 consecutive fine points (16 rows
// of 64 lanes, one point per lane per row) and keeps their sums in
// registers.  It walks the wavelength-sorted survivors whose centres lie
// within the point's largest half-window of its points, one record per lane
// (the next 64 prefetched while the current 64 are summed), tests their
// windows with one ballot, broadcasts each intersecting record with readlane
// and evaluates only the rows the window covers.  No atomics: each point is
// summed by one lane in the survivors' wavelength order, so results are
// bit-reproducible.  A line whose part is smooth over the whole tile
// (window over the tile, centre far outside it) is evaluated only at nodes
// of the tile, whose sums are interpolated at the end; in FP32 the farther
// such lines use fewer nodes, several lines to a 64-lane pass.
//
// Re w is evaluated in real arithmetic only, so that its relative accuracy
// holds where Re w << |w| (far wings of weakly damped lines):
//  - away from the core, a Gauss-Hermite quadrature of
//    H = (a/pi) int exp(-t^2) / ((x - t)^2 + a^2) dt, written as one fraction
//    of positive terms (nodes and weights computed at plan time);
//  - near the core, the trapezoidal rule for the same integral with the
//    contribution of the integrand's pole at t = x + i a added in closed
//    form (the error of the corrected rule is of order exp(-pi^2/h^2)); the
//    node grid is shifted by half a step when x lies near a node;
//  - near the core of weakly damped lines (FP32, a < 0.4), the Taylor series
//    of Re w in a, whose odd terms are derivatives of Dawson's function
//    (tabulated at plan time), plus the Gaussian e^{a^2 - x^2} cos 2xa.
// Each row of 64 points takes one of these forms for all its lanes, chosen
// from the smallest |x| in the row, so the wave never diverges.
// Mixed precision uses FP32 with Kahan-compensated sums (every summand is
// positive, so the compensated error bound is relative to the sum); the
// plain path uses FP64 throughout.
#include "odf_internal.h"

namespace odf {

namespace {

constexpr float kPiF = 3.14159265358979323846f;

// Workgroup order.  The hardware deals consecutive workgroups round-robin
// to the 8 XCDs, so consecutive tiles of a point land on different XCDs and
// every XCD gets an equal share of every point.  (Giving each XCD a
// contiguous range of points instead would let one expensive point -- costs
// differ by two orders of magnitude across the T-P grid -- idle the other
// XCDs.  Runs of 8 neighbouring tiles per XCD, for L2 sharing of the
// records they read, measured no change in time or in HBM reads: the
// records that concurrently resident workgroups stream exceed the L2 either
// way.)
__device__ __forceinline__ int tile_order(int bid, int total) {
  (void)total;
  return bid;
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

// Four-node Gauss-Hermite pair sum, valid to 2e-5 relative for |z| >= 6.
__device__ __forceinline__ float ring32(float x, float y, const QuadConsts* __restrict__ Q) {
  const float x2 = x * x, r2 = fmaf(y, y, x2);
  const float p1 = r2 + Q->gh4_t2[0], p2 = r2 + Q->gh4_t2[1];
  const float d1 = fmaf(p1, p1, -4.0f * Q->gh4_t2[0] * x2);
  const float d2 = fmaf(p2, p2, -4.0f * Q->gh4_t2[1] * x2);
  const float num = fmaf(Q->gh4_w[0] * p1, d2, Q->gh4_w[1] * p2 * d1);
  return 2.0f * y * num * __builtin_amdgcn_rcpf(d1 * d2);
}

// Pole-corrected trapezoidal rule, nodes t_k = (k + delta) h, for y < 6 and
// |x| up to about 30 (the running product is renormalised once so that it
// stays inside the FP32 range).  The node k = kTrap32Half lies beyond the
// rule's |t| <= kTrap32Tmax in both grids (weight zero), so the loop stops
// before it.
static_assert((float)kTrap32Half * kTrap32H > kTrap32Tmax, "last FP32 trapezoid node has weight zero");
__device__ __forceinline__ float core32(float x, float y, const QuadConsts* __restrict__ Q) {
  constexpr float h = kTrap32H;
  constexpr float invh = 1.0f / kTrap32H;
  const float y2 = y * y;
  const float hx = x * invh;
  const float fr = hx - rintf(hx);
  const bool sh = fabsf(fr) < 0.25f;
  const float xs = sh ? x - 0.5f * h : x;   // x - delta h: node k then sits at k h
  float num = 0.0f, den = 1.0f;
#pragma unroll
  for (int k = -kTrap32Half; k < kTrap32Half; ++k) {
    const float dd = xs - (float)k * h;
    const float D = fmaf(dd, dd, y2);
    const float ck = sh ? Q->tr32_ch[k + kTrap32Half] : Q->tr32_ci[k + kTrap32Half];
    num = fmaf(num, D, ck * den);
    den *= D;
    if (k == 0) {
      const float sc = den > 1.0e18f ? 1.0e-18f : 1.0f;
      num *= sc;
      den *= sc;
    }
  }
  float v = y * num * __builtin_amdgcn_rcpf(den);
  if (y < kPiF * invh) {
    // Re[ 2 e^{-z^2} / (1 -/+ e^{-2 pi i z / h}) ] with E = e^{-2 pi y/h} e^{2 pi i x/h};
    // the hardware sine and cosine take their argument in revolutions
    const float e2 = 2.0f * kPiF * y * invh;
    const float mag = __expf(y2 - x * x - e2);
    const float ep = __expf(-e2);
    const float ph = hx - rintf(hx);
    const float th0 = hx - x * y * (1.0f / kPiF);
    const float th = th0 - rintf(th0);
    const float sph = __builtin_amdgcn_sinf(ph), cph = __builtin_amdgcn_cosf(ph);
    const float sth = __builtin_amdgcn_sinf(th), cth = __builtin_amdgcn_cosf(th);
    const float sgn = sh ? 1.0f : -1.0f;
    const float dre = fmaf(ep, cph, sgn), dim = ep * sph;
    v += 2.0f * mag * fmaf(cth, dre, sth * dim) * __builtin_amdgcn_rcpf(fmaf(dre, dre, dim * dim));
  }
  return v;
}

// Small-damping series (a < 0.4) for every x:
//   H = e^{a^2 - x^2} cos(2 x a) + a sum_{k < nt} a^{2k} T_{2k+1}(x),
// with T_n read from the cubic table in LDS at s = 1/(1 + x^2).  The number
// of terms nt is chosen per line from a (series32_terms); relative error
// below 1e-5 including the FP32 table (truncation dominates near a = 0.4).
__device__ __forceinline__ int series32_terms(float y) {
  return y < 0.004f ? 1 : (y < 0.06f ? 2 : (y < 0.2f ? 3 : 4));
}

__device__ __forceinline__ float series32(float x, float y, float y2, float y_over_pi, int nt,
                                          const float4* __restrict__ tab) {
  const float x2 = x * x;
  const float t = __builtin_amdgcn_rcpf(1.0f + x2) * (float)kSerIntervals;
  const int i = min((int)t, kSerIntervals - 1);
  const float f = t - (float)i;
  const float4* __restrict__ c = tab + i;
  auto term = [&](int k) {
    const float4 q = c[k * kSerIntervals];
    return fmaf(fmaf(fmaf(q.w, f, q.z), f, q.y), f, q.x);
  };
  float U;
  if (nt == 4) U = fmaf(fmaf(fmaf(term(3), y2, term(2)), y2, term(1)), y2, term(0));
  else if (nt == 3) U = fmaf(fmaf(term(2), y2, term(1)), y2, term(0));
  else if (nt == 2) U = fmaf(term(1), y2, term(0));
  else U = term(0);
  // cos(2 x a): the hardware cosine takes revolutions, reduced to [-1/2, 1/2]
  const float r0 = x * y_over_pi;
  const float g = __expf(y2 - x2) * __builtin_amdgcn_cosf(r0 - rintf(r0));
  return fmaf(y, U, g);
}

// Per-line constants of the evaluation in u = sigma x (the record's far-wing
// fraction, with sigma folded into c1):
//   u(d) = d (c1 + c2 d + c3 d^2), c2 = c1 ln q / 2, c3 = c1 (ln q)^2 / 6,
//   u(row + 1) = u(row) q^-64 + step  (the frequency ratio of 64 points).
struct Far32 {
  float c1, c2, c3, step;
  float A, B, D, E;
};

// Bit mask of the rows (of the wave's 16) that meet [J - half, J + half].
__device__ __forceinline__ unsigned zone_rows(int J, int half, int t_lo) {
  if (half < 0) return 0u;
  const int a = J - half - t_lo, b = J + half - t_lo;
  if (b < 0 || a > kWavePoints - 1) return 0u;
  const int lo = max(a, 0) >> 6, hi = min(b, kWavePoints - 1) >> 6;
  return ((2u << hi) - 1u) & ~((1u << lo) - 1u);
}

// The wave's 16 row partial sums as one vector of registers.  Rows summed
// lane by lane are picked by a uniform runtime index, which indexes the
// register file directly (no LDS round trip per row, no LDS array for it).
typedef float RowVec __attribute__((ext_vector_type(kRows)));
static_assert(kRows == 16, "row partial sums are a 16-wide register vector");

__device__ __forceinline__ float far_value(float u, const Far32& f) {
  const float v = fmaf(u, u, f.D);
  return fmaf(v, f.A, f.B) * __builtin_amdgcn_rcpf(fmaf(v, v, f.E));
}

__device__ __forceinline__ float x_of_d32(float d, const Far32& f) {
  return d * fmaf(d, fmaf(d, f.c3, f.c2), f.c1);
}

// Far rows wholly inside the window, given as a bit mask of the wave's 16
// rows (all 16 when the window covers the tile and no row is near the core).
// Rows go in groups of eight: u is taken from the index at the start of a
// group and carried to the next row by the exact frequency ratio q^-64 (one
// FMA; the rounding this accumulates over seven rows stays below 1e-6 of
// u).  A row of a group that is not in the mask gets E = +inf (a scalar
// select), so its reciprocal is exactly zero and it adds nothing, at no extra
// vector cost (skipping such rows with a uniform branch per row instead
// measured 24 % slower overall); groups with no row in the mask are skipped.
__device__ __forceinline__ void rows32(unsigned rows, float d0, float q64, const Far32& f,
                                       RowVec& p) {
  constexpr int kGroup = 8;
  const int inf = 0x7f800000;
#pragma unroll
  for (int g = 0; g < kRows; g += kGroup) {
    const unsigned gm = (rows >> g) & ((1u << kGroup) - 1u);
    if (!gm) continue;
    float u = x_of_d32(d0 - (float)(64 * g), f);
#pragma unroll
    for (int r = 0; r < kGroup; ++r) {
      const int E = ((gm >> r) & 1u) ? __float_as_int(f.E) : inf;   // uniform
      const float v = fmaf(u, u, f.D);
      const float den = fmaf(v, v, __int_as_float(E));
      p[g + r] = fmaf(fmaf(v, f.A, f.B), __builtin_amdgcn_rcpf(den), p[g + r]);
      u = fmaf(u, q64, f.step);
    }
  }
}

// Row masks of 64 records at once, one record per lane, on the vector unit
// (one pass per batch of records instead of scalar work per line and wave):
//   rows  the tile's rows that the window meets
//   edge  rows cut by the window edge (it starts inside its first row or
//         ends inside its last)
//   near  rows meeting the |x| < 15 zone, core rows meeting |x| < 6
// Packed as far | (masked << 16) and near_in_window | (core << 16), where far
// are the rows summed in registers and masked those summed lane by lane.
// For records that meet the tile 0 <= jl <= jh <= 1023; the other lanes
// compute values that nobody reads.  A zone half-width of -32768 gives no
// rows.  A record whose window covers the tile, whose |x| < 15 zone misses
// it and whose centre lies more than kFFDist points outside the tile's 1024
// points is a far-field record: fm = nc = 0 and tier 1 to 4 by the centre's
// distance (beyond kFFDist, kFFTier2, kFFTier3, kFFTier4); tier 0 for the
// others.
__device__ __forceinline__ unsigned zone_rows_v(int rel, int z) {
  const int lo = min(max((rel - z) >> 6, 0), kRows);
  const int hi = min(max((rel + z) >> 6, -1), kRows - 1);
  return (0xffffu << lo) & (0xffffu >> (kRows - 1 - hi));
}

__device__ __forceinline__ void row_masks(int2 w, int2 jz, int t_lo, int t_hi, unsigned& fm,
                                          unsigned& nc, int& tier) {
  const int jl = max(w.x, t_lo) - t_lo;
  const int jh = min(w.y, t_hi) - t_lo;
  const int r_lo = (jl >> 6) & 31, r_hi = (jh >> 6) & 31;
  const unsigned rows = (0xffffu << r_lo) & (0xffffu >> ((kRows - 1 - r_hi) & 31));
  const unsigned edge = ((jl & 63) ? (1u << r_lo) : 0u) | ((jh & 63) != 63 ? (1u << r_hi) : 0u);
  const int rel = jz.x - t_lo;
  const unsigned near = zone_rows_v(rel, (int)(short)(jz.y & 0xffff));
  const unsigned core = zone_rows_v(rel, jz.y >> 16);
  fm = (rows & ~(near | edge)) | (((near | edge) & rows) << 16);
  nc = (near & rows) | (core << 16);
  const int dist = max(-rel, rel - (kWavePoints - 1));
  const bool far_field = w.x <= t_lo && w.y >= t_hi && near == 0u && dist > kFFDist;
  tier = 0;
  if (far_field) {
    fm = 0u;
    nc = 0u;
    tier = 1 + (dist > kFFTier2) + (dist > kFFTier3) + (dist > kFFTier4);
  }
}

__device__ __forceinline__ void line32(const Rec32& l, unsigned far_masked, unsigned near_core,
                                       int t_lo, int lane,
                                       float lnq2, float lnq6, float q64, float g64,
                                       const QuadConsts* __restrict__ Q, const float4* __restrict__ tab,
                                       RowVec& p) {
  Far32 f;
  f.c1 = l.c1;
  f.c2 = l.c1 * lnq2;
  f.c3 = l.c1 * lnq6;
  f.step = g64 * l.c1;
  f.A = l.A;
  f.B = l.B;
  f.D = l.D;
  f.E = l.E;
  const int rel = l.J - t_lo;
  const int ib = rel - lane;
  const float d0 = (float)ib + l.phi;
  // far rows in registers; edge rows and rows near the core lane by lane
  // (lanes past the grid's end are summed like the others and never stored)
  rows32(far_masked & 0xffffu, d0, q64, f, p);
  unsigned m = far_masked >> 16;
  if (!m) return;
  // per-lane masks, into the same register partial sums, row picked by its
  // index (near rows exist only for a < 15, where sigma = 1 and u = x)
  const unsigned nearr = near_core & 0xffffu;   // rows meeting |x| < 15
  const unsigned core = near_core >> 16;        // rows meeting |x| < 6
  const float y = l.y, S = l.S;
  const float y2 = y * y;
  const bool ser = y < kSerYMax;
  const int nt = series32_terms(y);
  const float y_over_pi = y * (1.0f / kPiF);
  while (m) {
    const int rr = __builtin_ctz(m);
    m &= m - 1u;
    const float d = (float)(ib - 64 * rr) + l.phi;   // exact near the centre
    const float x = x_of_d32(d, f);
    float v;
    if ((nearr >> rr) & 1u) {
      if ((core >> rr) & 1u) v = S * (ser ? series32(x, y, y2, y_over_pi, nt, tab) : core32(x, y, Q));
      else v = S * ring32(x, y, Q);
    } else {
      v = far_value(x, f);
    }
    const int j = t_lo + 64 * rr + lane;
    v = (j >= l.jlo && j <= l.jhi) ? v : 0.0f;
    p[rr] += v;
  }
}

// A nearest-tier far-field record (broadcast in scalar registers) at this
// lane's quarter node, at offset ffoff after the tile's first point.
__device__ __forceinline__ float far_node32(const Rec32& l, int t_lo, float ffoff, float lnq2,
                                            float lnq6) {
  Far32 f;
  f.c1 = l.c1;
  f.c2 = l.c1 * lnq2;
  f.c3 = l.c1 * lnq6;
  f.step = 0.0f;
  f.A = l.A;
  f.B = l.B;
  f.D = l.D;
  f.E = l.E;
  const float d = (float)(l.J - t_lo) + l.phi - ffoff;
  return far_value(x_of_d32(d, f), f);
}

// The far-field records of one whole-tile tier among the current 64 (bit
// mask mt, lane k holding record r_own), K nodes over the tile and 64 / K
// records per pass: lane group g = lane / K takes the g-th record of the
// pass at node lane % K (offset off).  The records' indices go through an
// LDS queue in lane order; each lane then reads its record's fields with
// vector loads.  Returns this lane's sum over the passes (at most 64 / (64
// / K) = K terms, added plainly).
template <int K>
__device__ __forceinline__ float far_tier32(unsigned long long mt, int r_own, int lane, int t_lo,
                                            float off, int* __restrict__ q,
                                            const Rec32* __restrict__ rec, float lnq2, float lnq6) {
  constexpr int kShift = K == 32 ? 5 : (K == 16 ? 4 : 3);
  static_assert((1 << kShift) == K, "tiers of 32, 16 or 8 nodes");
  if ((mt >> lane) & 1ull) {
    const unsigned rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mt >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((unsigned)mt, 0u));
    q[rank] = r_own;
  }
  __builtin_amdgcn_wave_barrier();
  const int cnt = __popcll(mt);
  const int g = lane >> kShift;
  float acc = 0.0f;
  for (int p = 0; p < cnt; p += 64 / K) {
    // lanes past the last record read the last one again and add nothing
    const int qi = p + g;
    const int r = q[min(qi, cnt - 1)];
    const int* __restrict__ w = reinterpret_cast<const int*>(rec + r);
    const int J = w[0];
    const float4 a = *reinterpret_cast<const float4*>(w + 4);   // phi, c1, A, B
    const float2 b = *reinterpret_cast<const float2*>(w + 8);   // D, E
    Far32 f;
    f.c1 = a.y;
    f.c2 = a.y * lnq2;
    f.c3 = a.y * lnq6;
    f.step = 0.0f;
    f.A = a.z;
    f.B = a.w;
    f.D = b.x;
    f.E = b.y;
    const float d = (float)(J - t_lo) + a.x - off;
    const float v = far_value(x_of_d32(d, f), f);
    acc += qi < cnt ? v : 0.0f;
  }
  __builtin_amdgcn_wave_barrier();
  return acc;
}

// v, made opaque to the optimiser: a load indexed by it stays where it is
// written instead of being hoisted out of the record loop, where its result
// would hold a register through the line loop (which has none to spare).
__device__ __forceinline__ int opaque(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Per-wave LDS: the row sums' compensations, the far-field sums and the
// record queue.
struct WaveLds32 {
  // Kahan compensations of the 16 row sums, two to a word as the upper 16
  // bits of the FP32 value (8 significant bits): a compensation is at most
  // about an ulp of its sum, so truncating it loses at most 2^-8 ulp per
  // flush
  unsigned rc[kRows / 2][kWave];
  // far-field sums and their compensations: [0] the quarter nodes (lane l
  // at node l % 16 of quarter l / 16), [1..3] the lane slots of the 32-,
  // 16- and 8-node tiers (lane l at node l % K of lane group l / K)
  float fs[4][kWave];
  float fc[4][kWave];
  // one tier's record queue; at the end the whole-tile tiers' node values
  int q[kWave];
};

__device__ __forceinline__ void kahan_lds(float* __restrict__ s, float* __restrict__ c, int lane,
                                          float v) {
  float sum = s[lane], cc = c[lane];
  kahan_add(sum, cc, v);
  s[lane] = sum;
  c[lane] = cc;
}

// Compensated (Kahan) addition of the partial sums into the row sums: the
// running sums s stay in registers, their compensations in LDS.
__device__ __forceinline__ void flush32(float (&s)[kRows], RowVec& p, unsigned* __restrict__ rc,
                                        int lane) {
#pragma unroll
  for (int i = 0; i < kRows / 2; ++i) {
    const int o = i * 64 + lane;
    const unsigned w = rc[o];
    float c0 = __uint_as_float(w << 16), c1 = __uint_as_float(w & 0xffff0000u);
    kahan_add(s[2 * i], c0, p[2 * i]);
    kahan_add(s[2 * i + 1], c1, p[2 * i + 1]);
    rc[o] = (__float_as_uint(c0) >> 16) | (__float_as_uint(c1) & 0xffff0000u);
    p[2 * i] = 0.0f;
    p[2 * i + 1] = 0.0f;
  }
}

// The far field at point k (0..255) of a quarter from its 16 node values
// (barycentric formula for Chebyshev points of the first kind; no point of
// the quarter coincides with a node: the closest is 2.2e-5 away in t).
__device__ __forceinline__ float far_field_at(const float* __restrict__ nodes, int k,
                                              const QuadConsts* __restrict__ Q) {
  const float t = ((float)k - 127.5f) * (1.0f / 127.5f);
  float num = 0.0f, den = 0.0f;
#pragma unroll
  for (int n = 0; n < kFFNodes; ++n) {
    const float r = Q->ff_w[n] * __builtin_amdgcn_rcpf(t - Q->ff_s[n]);
    num = fmaf(r, nodes[n], num);
    den += r;
  }
  return num / den;
}

// A whole record with one scalar-memory wait.  Left to itself the compiler
// loads each field where it is first used, behind the branches of the line
// routine, and waits for scalar memory three times per line; the empty asm
// that takes all twelve words in scalar registers puts the loads and their
// single wait here.
__device__ __forceinline__ Rec32 load_rec32(const Rec32* __restrict__ p) {
  // read through the constant address space: the records are not written
  // while the kernel runs, and a uniform constant load is always a scalar
  // load (a global one only when the compiler proves nothing clobbers it)
  typedef int v4i __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(4))) v4i cv4i;
  const cv4i* q = (const cv4i*)p;
  const v4i a = q[0], b = q[1], c = q[2];
  asm volatile("" ::"s"(a.x), "s"(a.y), "s"(a.z), "s"(a.w), "s"(b.x), "s"(b.y), "s"(b.z), "s"(b.w),
               "s"(c.x), "s"(c.y), "s"(c.z), "s"(c.w));
  Rec32 r;
  r.J = a.x;
  r.jlo = a.y;
  r.jhi = a.z;
  r.czh = a.w;
  r.phi = __int_as_float(b.x);
  r.c1 = __int_as_float(b.y);
  r.A = __int_as_float(b.z);
  r.B = __int_as_float(b.w);
  r.D = __int_as_float(c.x);
  r.E = __int_as_float(c.y);
  r.S = __int_as_float(c.z);
  r.y = __int_as_float(c.w);
  return r;
}

// lines summed in plain FP32 between two compensated additions (the plain
// partial of at most 64 positive terms is within 64 u = 3.8e-6 of its value)
constexpr int kFlushLines = 64;

// Six workgroups per CU (6 waves per SIMD): at most 80 VGPRs, which the
// register allocator meets without spilling, and 24 KB of LDS per workgroup.
// It measured 5 % faster than the 5 waves per SIMD that 95 VGPRs give.
__global__ __launch_bounds__(256, 6) void k_voigt32(Params P, Batch B,
                                                    const QuadConsts* __restrict__ Q,
                                                    int tiles_per_point, int total) {
  __shared__ WaveLds32 lds_w[kWavesPerWG];
  __shared__ float4 lds_ser[kSerTerms * kSerIntervals]; // small-damping series table
  __shared__ float lds_toff[kFFTileNodes];               // whole-tile tier node positions
  const int logical = tile_order(blockIdx.x, total);
  if (logical >= total) return;
  {
    const float4* __restrict__ src = reinterpret_cast<const float4*>(&Q->ser[0][0][0]);
    for (int i = threadIdx.x; i < kSerTerms * kSerIntervals; i += blockDim.x) lds_ser[i] = src[i];
    if (threadIdx.x < kFFTileNodes) lds_toff[threadIdx.x] = Q->ff_toff[threadIdx.x];
    __syncthreads();
  }
  const int pt = logical / tiles_per_point;
  const int tile = logical - pt * tiles_per_point;
  // wave index is uniform across the wave; say so, so that everything derived
  // from the tile origin stays in scalar registers and branches stay scalar
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = (int)P.N;
  const int t_lo = tile * kWGPoints + wid * kWavePoints;
  if (t_lo >= N) return;
  const int t_hi = min(t_lo + kWavePoints - 1, N - 1);
  WaveLds32& L = lds_w[wid];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    L.fs[k][lane] = 0.0f;
    L.fc[k][lane] = 0.0f;
  }
  unsigned ffmask = 0u;   // far-field tiers seen (bit t - 1 for tier t)
  float s[kRows];
  RowVec p;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    s[rr] = 0.0f;
    p[rr] = 0.0f;
  }
#pragma unroll
  for (int i = 0; i < kRows / 2; ++i) L.rc[i][lane] = 0u;
  const Rec32* __restrict__ rec = reinterpret_cast<const Rec32*>(B.rec) + pt * B.rec_stride;
  const int2* __restrict__ win = B.win + pt * B.rec_stride;
  const int2* __restrict__ wz = B.wz + pt * B.rec_stride;
  const int ns = B.nsurv[pt];
  const int nn = B.nsurv_n[pt];
  const float lnq = (float)P.lnq;
  const float lnq2 = lnq * 0.5f, lnq6 = lnq * lnq * (1.0f / 6.0f);
  const float q64 = (float)exp(-64.0 * P.lnq);              // nu(j + 64) / nu(j)
  const float g64 = (float)(expm1(-64.0 * P.lnq) / P.lnq);  // (q^-64 - 1) / ln q
  int since_flush = 0;
  // the narrow class, then the wide one, each scanned over the records whose
  // centres lie within that class's largest half-window of the tile: one
  // loop over a virtual index v that runs through both ranges, record
  // c0n + v below n1 and c0n + v + shift from there on
  const int Hn = B.hmax[pt], Hw = B.hmax_w[pt];
  const int c0n = lower_bound_J(rec, nn, t_lo - Hn), c1n = upper_bound_J(rec, nn, t_hi + Hn);
  const int c0w = nn + lower_bound_J(rec + nn, ns - nn, t_lo - Hw);
  const int c1w = nn + upper_bound_J(rec + nn, ns - nn, t_hi + Hw);
  const int n1 = c1n - c0n, nv = n1 + (c1w - c0w);
  const int shift = c0w - c0n - n1;
  // the windows of 64 records (from the compact window array), one per
  // lane, the next 64 prefetched while these are summed; each intersecting
  // record is then read with scalar loads
  // (lanes past the end hold an empty window that meets no tile)
  const int2 none = make_int2(0x3fffffff, -0x3fffffff);
  int2 nxt = none, nxz = make_int2(0, 0);
  if (lane < nv) {
    const int r = c0n + lane + (lane >= n1 ? shift : 0);
    nxt = win[r];
    nxz = wz[r];
  }
  for (int vb = 0; vb < nv; vb += 64) {
    const int2 cur = nxt, cz = nxz;
    nxt = none;
    const int vn = vb + 64 + lane;
    if (vn < nv) {
      const int r = c0n + vn + (vn >= n1 ? shift : 0);
      nxt = win[r];
      nxz = wz[r];
    }
    unsigned long long m = __ballot(cur.x <= t_hi && cur.y >= t_lo);
    if (!m) continue;
    unsigned fm, nc;
    int tier;
    row_masks(cur, cz, t_lo, t_hi, fm, nc, tier);
    // far-field records in loops of their own (a branch between the two
    // kinds inside one loop costs the row sums' registers spills): the
    // nearest tier one record at a time at the quarter nodes, the others
    // several to a pass
    unsigned long long mf = m & __ballot(tier == 1);
    const unsigned long long m2 = m & __ballot(tier == 2);
    const unsigned long long m3 = m & __ballot(tier == 3);
    const unsigned long long m4 = m & __ballot(tier == 4);
    m &= ~(mf | m2 | m3 | m4);
    if (mf) {
      ffmask |= 1u;
      const float ffoff = Q->ff_off[opaque(lane)];
      float acc = 0.0f;
      while (mf) {
        const int k = __builtin_amdgcn_readfirstlane(__builtin_ctzll(mf));
        mf &= mf - 1;
        const int r = c0n + vb + k + (vb + k >= n1 ? shift : 0);
        acc += far_node32(load_rec32(rec + r), t_lo, ffoff, lnq2, lnq6);
      }
      kahan_lds(L.fs[0], L.fc[0], lane, acc);
    }
    if (m2 | m3 | m4) {
      const int r_own = c0n + vb + lane + (vb + lane >= n1 ? shift : 0);
      if (m2) {
        ffmask |= 2u;
        kahan_lds(L.fs[1], L.fc[1], lane,
                  far_tier32<32>(m2, r_own, lane, t_lo, lds_toff[opaque(lane) & 31], L.q, rec, lnq2, lnq6));
      }
      if (m3) {
        ffmask |= 4u;
        kahan_lds(L.fs[2], L.fc[2], lane,
                  far_tier32<16>(m3, r_own, lane, t_lo, lds_toff[32 + (opaque(lane) & 15)], L.q, rec, lnq2, lnq6));
      }
      if (m4) {
        ffmask |= 8u;
        kahan_lds(L.fs[3], L.fc[3], lane,
                  far_tier32<8>(m4, r_own, lane, t_lo, lds_toff[48 + (opaque(lane) & 7)], L.q, rec, lnq2, lnq6));
      }
    }
    while (m) {
      const int k = __builtin_amdgcn_readfirstlane(__builtin_ctzll(m));
      m &= m - 1;
      const int r = c0n + vb + k + (vb + k >= n1 ? shift : 0);
      line32(load_rec32(rec + r), __builtin_amdgcn_readlane(fm, k),
             __builtin_amdgcn_readlane(nc, k), t_lo, lane, lnq2, lnq6, q64, g64, Q, lds_ser, p);
      if (++since_flush == kFlushLines) {
        flush32(s, p, &L.rc[0][0], lane);
        since_flush = 0;
      }
    }
  }
  flush32(s, p, &L.rc[0][0], lane);
  // the far field at this lane's quarter node: the nearest tier's sum plus
  // each whole-tile tier's interpolant there; node values read by every lane
  // below
  if (ffmask) {
    float ff = L.fs[0][lane] - L.fc[0][lane];
    if (ffmask & 14u) {
      // node n of a tier with K nodes: the sum of its 64 / K lane slots
      float f = 0.0f;
      if (lane < 32) {
#pragma unroll
        for (int g = 0; g < 2; ++g) f += L.fs[1][32 * g + lane] - L.fc[1][32 * g + lane];
      } else if (lane < 48) {
#pragma unroll
        for (int g = 0; g < 4; ++g) f += L.fs[2][16 * g + lane - 32] - L.fc[2][16 * g + lane - 32];
      } else if (lane < kFFTileNodes) {
#pragma unroll
        for (int g = 0; g < 8; ++g) f += L.fs[3][8 * g + lane - 48] - L.fc[3][8 * g + lane - 48];
      }
      float* nodes = reinterpret_cast<float*>(L.q);
      nodes[lane] = f;
      __builtin_amdgcn_wave_barrier();
#pragma unroll 8
      for (int n = 0; n < kFFTileNodes; ++n) ff = fmaf(Q->ff_V[n][lane], nodes[n], ff);
      __builtin_amdgcn_wave_barrier();
    }
    L.fs[0][lane] = ff;
    __builtin_amdgcn_wave_barrier();
  }
  float* kap = reinterpret_cast<float*>(B.kappa) + pt * B.kappa_stride;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    const int j = t_lo + rr * 64 + lane;
    const unsigned w = L.rc[rr >> 1][lane];
    const float c = __uint_as_float((rr & 1) ? (w & 0xffff0000u) : (w << 16));
    const float v = s[rr] - c;
    const float ffv = ffmask ? far_field_at(L.fs[0] + kFFNodes * (rr >> 2), 64 * (rr & 3) + lane, Q) : 0.0f;
    if (j <= t_hi) kap[j] = v + ffv;
  }
}

// ---------------------------------------------------------------- FP64 ----

// 1/d for d > 0 in the normal range: the hardware approximation refined by
// two Newton steps, e = 1 - d r, r <- r + r e (the error squares each step,
// so the result is within about an ulp; no scaling or special cases needed).
// One Newton step: the hardware approximation is within 5e-8 relative
// (measured on gfx950 over 2^-60 .. 2^60), so one step leaves about 2e-15,
// far below the 5e-13 and 3e-12 of the Gauss-Hermite rules that use it.
__device__ __forceinline__ double rcp64_1(double d) {
  const double r = __builtin_amdgcn_rcp(d);
  return fma(r, fma(-d, r, 1.0), r);
}

__device__ __forceinline__ double rcp64(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = fma(-d, r, 1.0);
  r = fma(r, e, r);
  e = fma(-d, r, 1.0);
  return fma(r, e, r);
}

// Eight-node Gauss-Hermite pair sum for |z| >= 10 (relative error < 5e-13).
__device__ __forceinline__ double gh8(double x2, double y, double r2, const QuadConsts* __restrict__ Q) {
  const double p1 = r2 + Q->gh8_t2[0];
  const double d1 = fma(p1, p1, -4.0 * Q->gh8_t2[0] * x2);
  double num = Q->gh8_w[0] * p1, den = d1;
#pragma unroll
  for (int k = 1; k < 4; ++k) {
    const double pk = r2 + Q->gh8_t2[k];
    const double dk = fma(pk, pk, -4.0 * Q->gh8_t2[k] * x2);
    num = fma(num, dk, Q->gh8_w[k] * pk * den);
    den *= dk;
  }
  return 2.0 * y * num * rcp64_1(den);
}

// Four-node Gauss-Hermite pair sum for |z| >= 40 (relative error < 3e-12) as
// one fraction in X = x^2, times S:  S H = N(X) / D(X) with
//   d_k = (X + c_k)^2 - 4 t_k^2 X = X^2 + e_k X + c_k^2,  c_k = a^2 + t_k^2,
//   e_k = 2a^2 - 2t_k^2,  D = d_1 d_2 (monic quartic),
//   N = 2 a S (w_1 (X + c_1) d_2 + w_2 (X + c_2) d_1) (cubic).
// The coefficients are per line; a sample then costs two Horner chains and a
// reciprocal.  At |x| >= 40 the leading terms dominate the others by a factor
// of at least 300, so the expanded form keeps the rule's accuracy.
struct Gh4Frac {
  double a3, a2, a1, a0;   // numerator, highest power first
  double b3, b2, b1, b0;   // denominator without its leading 1
};

__device__ __forceinline__ Gh4Frac gh4_fraction(double y, double S, const QuadConsts* __restrict__ Q) {
  const double y2 = y * y;
  const double t1 = Q->gh4_t2d[0], t2 = Q->gh4_t2d[1];
  const double w1 = Q->gh4_wd[0], w2 = Q->gh4_wd[1];
  const double c1 = y2 + t1, c2 = y2 + t2;
  const double e1 = 2.0 * (y2 - t1), e2 = 2.0 * (y2 - t2);
  const double q1 = c1 * c1, q2 = c2 * c2;
  const double K = 2.0 * y * S;
  Gh4Frac f;
  f.b3 = e1 + e2;
  f.b2 = q1 + q2 + e1 * e2;
  f.b1 = e1 * q2 + e2 * q1;
  f.b0 = q1 * q2;
  f.a3 = K * (w1 + w2);
  f.a2 = K * (w1 * (e2 + c1) + w2 * (e1 + c2));
  f.a1 = K * (w1 * (q2 + c1 * e2) + w2 * (q1 + c2 * e1));
  f.a0 = K * (w1 * c1 * q2 + w2 * c2 * q1);
  return f;
}

__device__ __forceinline__ double gh4_value(double X, const Gh4Frac& f) {
  const double num = fma(fma(fma(f.a3, X, f.a2), X, f.a1), X, f.a0);
  const double den = fma(fma(fma(X + f.b3, X, f.b2), X, f.b1), X, f.b0);
  return num * rcp64_1(den);
}

// Pole-corrected trapezoidal rule (FP64), any x reached by a core row; ep is
// the line's e^{-2 pi a / h}.  As in FP32, the node k = kTrap64Half has
// weight zero in both grids and is left out.
static_assert(kTrap64Half * kTrap64H > kTrap64Tmax, "last FP64 trapezoid node has weight zero");
__device__ __forceinline__ double core64(double x, double y, double ep, const QuadConsts* __restrict__ Q) {
  constexpr double h = kTrap64H;
  constexpr double invh = 1.0 / kTrap64H;
  const double y2 = y * y;
  const double hx = x * invh;
  const double fr = hx - rint(hx);
  const bool sh = fabs(fr) < 0.25;
  const double xs = sh ? x - 0.5 * h : x;   // x - delta h: node k then sits at k h
  double num = 0.0, den = 1.0;
#pragma unroll
  for (int k = -kTrap64Half; k < kTrap64Half; ++k) {
    const double dd = xs - (double)k * h;
    const double D = fma(dd, dd, y2);
    const double ck = sh ? Q->tr64_ch[k + kTrap64Half] : Q->tr64_ci[k + kTrap64Half];
    num = fma(num, D, ck * den);
    den *= D;
  }
  double v = y * num * rcp64(den);
  if (y < kPi * invh) {
    const double e2 = 2.0 * kPi * y * invh;
    const double mag = exp(y2 - x * x - e2);
    double sph, cph, sth, cth;
    sincospi(2.0 * hx, &sph, &cph);
    sincospi(2.0 * hx - 2.0 * x * y / kPi, &sth, &cth);
    const double sgn = sh ? 1.0 : -1.0;
    const double dre = fma(ep, cph, sgn), dim = ep * sph;
    v += 2.0 * mag * (cth * dre + sth * dim) * rcp64(fma(dre, dre, dim * dim));
  }
  return v;
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

__device__ __forceinline__ void line64(const Rec64& l, int t_lo, int t_hi, int lane, double lnq,
                                       double q64, double g64, const QuadConsts* __restrict__ Q,
                                       double (&as)[kRows], double* __restrict__ ls) {
  const double y2 = l.y * l.y;
  const int ib = l.J - t_lo - lane;
  const int jl = max(l.jlo, t_lo) - t_lo;
  const int jh = min(l.jhi, t_hi) - t_lo;
  const int r_lo = jl >> 6, r_hi = jh >> 6;
  const unsigned rows = ((2u << r_hi) - 1u) & ~((1u << r_lo) - 1u);
  const unsigned core = zone_rows(l.J, l.czh, t_lo) & rows;
  const unsigned mid = zone_rows(l.J, l.z40, t_lo) & rows & ~core;
  const unsigned far = rows & ~core;
  // x from the index at the first row of each run of rows, then carried to
  // the next row by the exact frequency ratio q^-64 (one FMA)
  const double step = g64 * l.c1;
  Gh4Frac g4{};
  if (far & ~mid) g4 = gh4_fraction(l.y, l.S, Q);
  double x = 0.0;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    if (!(far & (1u << rr))) continue;
    if (rr == 0 || !((far >> (rr - 1)) & 1u)) x = x_of_d64((double)(ib - 64 * rr) + l.phi, l.c1, lnq);
    else x = fma(x, q64, step);
    const double x2 = x * x;
    double v = (mid >> rr) & 1u ? l.S * gh8(x2, l.y, x2 + y2, Q) : gh4_value(x2, g4);
    const int rs = t_lo + 64 * rr;
    if (rs < l.jlo || rs + 63 > l.jhi) {
      const int j = rs + opaque(lane);   // recomputed, not kept (and spilled) for all 16 rows
      v = (j >= l.jlo && j <= l.jhi) ? v : 0.0;
    }
    as[rr] += v;
  }
  unsigned m = core;
  if (!m) return;
  const double ep = exp(-2.0 * kPi * l.y / kTrap64H);
  while (m) {
    const int rr = __builtin_ctz(m);
    m &= m - 1u;
    const double d = (double)(ib - 64 * rr) + l.phi;
    const double x = x_of_d64(d, l.c1, lnq);
    double v = l.S * core64(x, l.y, ep, Q);
    const int j = t_lo + 64 * rr + lane;
    v = (j >= l.jlo && j <= l.jhi) ? v : 0.0;
    ls[rr * 64 + lane] += v;
  }
}

// A far-field record (FP64): its four-node fraction at this lane's node,
// added to the node's sum in LDS.
__device__ __forceinline__ void far_field64(const Rec64& l, int t_lo, int lane, double lnq,
                                            const QuadConsts* __restrict__ Q,
                                            double* __restrict__ lff) {
  const Gh4Frac g4 = gh4_fraction(l.y, l.S, Q);
  const double d = (double)(l.J - t_lo) + l.phi - Q->ff_off64[lane];
  const double x = x_of_d64(d, l.c1, lnq);
  lff[lane] += gh4_value(x * x, g4);
}

// A whole FP64 record with one scalar-memory wait (as load_rec32).
__device__ __forceinline__ Rec64 load_rec64(const Rec64* __restrict__ p) {
  const int4* q = reinterpret_cast<const int4*>(p);
  const int4 a = q[0], b = q[1], c = q[2], d = q[3];
  asm volatile("" ::"s"(a.x), "s"(a.y), "s"(a.z), "s"(a.w), "s"(b.x), "s"(b.y), "s"(c.x), "s"(c.y),
               "s"(c.z), "s"(c.w), "s"(d.x), "s"(d.y), "s"(d.z), "s"(d.w));
  Rec64 r;
  r.J = a.x;
  r.jlo = a.y;
  r.jhi = a.z;
  r.czh = a.w;
  r.z40 = b.x;
  r.li = b.y;
  r.pad0 = b.z;
  r.pad1 = b.w;
  r.phi = __hiloint2double(c.y, c.x);
  r.S = __hiloint2double(c.w, c.z);
  r.y = __hiloint2double(d.y, d.x);
  r.c1 = __hiloint2double(d.w, d.z);
  return r;
}

// Four workgroups per CU (4 waves per SIMD, at most 128 VGPRs): a few
// registers spill, and that measured 6 % faster than 3 waves without spills.
__global__ __launch_bounds__(256, 4) void k_voigt64(Params P, Batch B, const QuadConsts* __restrict__ Q,
                                                 int tiles_per_point, int total) {
  __shared__ double lds_s[kWavesPerWG][kWavePoints];
  __shared__ double lds_ff[kWavesPerWG][kWave];   // far-field node sums
  const int logical = tile_order(blockIdx.x, total);
  if (logical >= total) return;
  const int p = logical / tiles_per_point;
  const int tile = logical - p * tiles_per_point;
  // wave index is uniform across the wave; say so, so that everything derived
  // from the tile origin stays in scalar registers and branches stay scalar
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int N = (int)P.N;
  const int t_lo = tile * kWGPoints + wid * kWavePoints;
  if (t_lo >= N) return;
  const int t_hi = min(t_lo + kWavePoints - 1, N - 1);
  double* ls = lds_s[wid];
  double* lff = lds_ff[wid];
  lff[lane] = 0.0;
  bool any_ff = false;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) ls[rr * 64 + lane] = 0.0;
  double as[kRows];
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) as[rr] = 0.0;
  const Rec64* __restrict__ rec = reinterpret_cast<const Rec64*>(B.rec) + p * B.rec_stride;
  const int2* __restrict__ win = B.win + p * B.rec_stride;
  const int2* __restrict__ wz = B.wz + p * B.rec_stride;
  const int ns = B.nsurv[p];
  const int nn = B.nsurv_n[p];
  const double lnq = P.lnq;
  const double q64 = exp(-64.0 * lnq);              // nu(j + 64) / nu(j)
  const double g64 = expm1(-64.0 * lnq) / lnq;      // (q^-64 - 1) / ln q
  // the narrow class, then the wide one (one loop over both ranges, as in
  // k_voigt32)
  const int Hn = B.hmax[p], Hw = B.hmax_w[p];
  const int c0n = lower_bound_J(rec, nn, t_lo - Hn), c1n = upper_bound_J(rec, nn, t_hi + Hn);
  const int c0w = nn + lower_bound_J(rec + nn, ns - nn, t_lo - Hw);
  const int c1w = nn + upper_bound_J(rec + nn, ns - nn, t_hi + Hw);
  const int n1 = c1n - c0n, nv = n1 + (c1w - c0w);
  const int shift = c0w - c0n - n1;
  // windows and (J, z40) one per lane (next 64 prefetched), records by
  // scalar loads
  const int2 none = make_int2(0x7fffffff, -0x7fffffff - 1);
  int2 nxt = none, nxz = make_int2(0, -1);
  if (lane < nv) {
    const int r = c0n + lane + (lane >= n1 ? shift : 0);
    nxt = win[r];
    nxz = wz[r];
  }
  for (int vb = 0; vb < nv; vb += 64) {
    const int2 cur = nxt, cz = nxz;
    nxt = none;
    const int vn = vb + 64 + lane;
    if (vn < nv) {
      const int r = c0n + vn + (vn >= n1 ? shift : 0);
      nxt = win[r];
      nxz = wz[r];
    }
    unsigned long long m = __ballot(cur.x <= t_hi && cur.y >= t_lo);
    if (!m) continue;
    // far field: window over the tile, |x| < 40 zone outside it, centre more
    // than kFFDist64 points away
    const int rel = cz.x - t_lo;
    const bool ff = cur.x <= t_lo && cur.y >= t_hi &&
                    (cz.y < 0 || cz.x + cz.y < t_lo || cz.x - cz.y > t_hi) &&
                    (rel < -kFFDist64 || rel > kWavePoints - 1 + kFFDist64);
    unsigned long long mf = m & __ballot(ff);
    m &= ~mf;
    if (mf) any_ff = true;
    while (mf) {
      const int k = __builtin_amdgcn_readfirstlane(__ffsll((long long)mf) - 1);
      mf &= mf - 1;
      const int r = c0n + vb + k + (vb + k >= n1 ? shift : 0);
      far_field64(load_rec64(rec + r), t_lo, lane, lnq, Q, lff);
    }
    while (m) {
      const int k = __builtin_amdgcn_readfirstlane(__ffsll((long long)m) - 1);
      m &= m - 1;
      const int r = c0n + vb + k + (vb + k >= n1 ? shift : 0);
      line64(load_rec64(rec + r), t_lo, t_hi, lane, lnq, q64, g64, Q, as, ls);
    }
  }
  double* kap = reinterpret_cast<double*>(B.kappa) + p * B.kappa_stride;
#pragma unroll
  for (int rr = 0; rr < kRows; ++rr) {
    const int j = t_lo + rr * 64 + lane;
    double w = 0.0;
    if (any_ff) {
      // point 64 (rr % 4) + lane of quarter rr / 4 from that quarter's nodes
      const double* __restrict__ M = Q->ff_M64[64 * (rr & 3) + lane];
      const double* __restrict__ f = lff + kFFNodes * (rr >> 2);
#pragma unroll
      for (int n = 0; n < kFFNodes; ++n) w = fma(M[n], f[n], w);
    }
    if (j <= t_hi) kap[j] = as[rr] + ls[rr * 64 + lane] + w;
  }
}

}  // namespace

hipError_t launch_voigt(hipStream_t st, const Params& P, const Batch& B, const QuadConsts* __restrict__ Q) {
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

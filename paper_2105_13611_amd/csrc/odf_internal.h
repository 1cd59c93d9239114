// Internal layout shared by the host runtime and the gfx950 kernels of the
// ODF engine.  Nothing here is part of the public C ABI (include/odf.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace odf {

// ---- physical constants, CGS (CODATA 2018) --------------------------------
constexpr double kC = 2.99792458e10;           // cm/s
constexpr double kH = 6.62607015e-27;          // erg s
constexpr double kK = 1.380649e-16;            // erg/K
constexpr double kEcharge = 4.803204712570263e-10;  // statC
constexpr double kMe = 9.1093837015e-28;       // g
constexpr double kAmu = 1.66053906660e-24;     // g
constexpr double kEv = 1.602176634e-12;        // erg
constexpr double kMassH = 1.008;               // amu
constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.77245385090551602730;

// ---- tiling of the Voigt scatter-sum --------------------------------------
constexpr int kWave = 64;
constexpr int kRows = 16;                        // rows of 64 points per wave
constexpr int kWavePoints = kWave * kRows;       // 1024 fine points per wave
constexpr int kWavesPerWG = 4;
constexpr int kWGPoints = kWavePoints * kWavesPerWG;  // 4096 per workgroup
constexpr int kLineBlock = 256;                  // lines per workgroup in K1
// Survivors are emitted in two classes by half-window (the larger of the
// two sides, in fine points): narrow (at most kNarrowHalf) first, then wide,
// each class in wavelength order.  A Voigt wave scans each class only
// within that class's largest half-window of its tile, so the thousands of
// narrow lines around a tile are not scanned out to the reach of the few
// capped lines whose windows span thousands of points.
constexpr int kNarrowHalf = 1024;
constexpr int kMaxBatch = 64;                    // points per device batch (bit masks in K1)

// ---- Voigt region constants -----------------------------------------------
// FP32: rows of 64 fine points are classified by the smallest |x| in them:
// all |x| >= 15 -> two-node Gauss-Hermite pair; all |x| >= 6 -> four-node;
// otherwise the pole-corrected trapezoidal rule (h = 0.75, nodes |t| <= 4.2)
// for every lane of the row.
constexpr float kFarR32 = 15.0f;
constexpr float kRingR32 = 6.0f;
constexpr int kTrap32Half = 6;                   // k = -6..6
constexpr float kTrap32H = 0.75f;
constexpr float kTrap32Tmax = 4.2f;
// FP64: rows with all |x| >= 40 -> four-node Gauss-Hermite pair sum (relative
// error below 3e-12); all |x| >= 8 -> eight-node (below 2e-11, 4e-13 from
// |x| = 10 on); other rows -> trapezoid h = 0.55, nodes |t| <= 5.9 (below
// 1.2e-13), for every lane.
constexpr double kFarR64 = 8.0;
constexpr double kFar4R64 = 40.0;
constexpr int kTrap64Half = 11;                  // k = -11..11
constexpr double kTrap64H = 0.55;
constexpr double kTrap64Tmax = 5.9;

// FP32 small-damping form for rows near the core of lines with a < 0.4:
//   H(x, a) = e^{a^2 - x^2} cos(2 x a) + sum_k a^{2k+1} T_{2k+1}(x),
//   T_n(x) = (-1)^{(n+1)/2} (2/sqrt(pi)) F^(n)(x) / n!,  F = Dawson's function,
// the Taylor series in a of Re w(x + i a), with k < kSerTerms terms.  Each
// T_n is tabulated against s = 1/(1 + x^2) in (0, 1] (all x) as one cubic per
// interval of width 1/kSerIntervals.
constexpr float kSerYMax = 0.4f;
constexpr int kSerTerms = 4;
constexpr int kSerIntervals = 128;

// FP32 far field of a tile: a line whose window covers the wave's whole tile,
// whose |x| < 15 zone misses it and whose centre lies more than kFFDist
// points outside it adds a smooth function of the grid index to the tile.
// Such lines are evaluated only at kFFNodes Chebyshev points (first kind) in
// each quarter of the tile, one per lane, and their sum is interpolated to
// the tile's points at the end.  The poles of a line's two-node fraction lie
// within sqrt(a^2 + 1/2) Doppler widths of its centre (in the complex plane;
// off the real axis for large a), and the centre is more than kFFDist points
// and more than 15 Doppler widths from the tile, so every pole is at least
// 0.9 kFFDist = 58 points outside it: at least 186 points from the middle
// of the nearest 256-point quarter (half-length 128), so the interpolation
// converges like rho^-16, rho = s + sqrt(s^2 - 1), s = 186/128, times a
// factor of order 16 for the double pole of the far wing.  In float64 the
// error at the rule's edge stays below 1.4e-5 of that line's part (damping
// 1e-4 to 1e5, Doppler widths of 1 to 60 points); the two-node fraction
// itself is within 5e-5 of H at |x| = 15.
constexpr int kFFNodes = 16;
constexpr int kFFQuarter = 256;
constexpr int kFFDist = 64;
// Distance tiers of the FP32 far field.  Farther lines are smoother over the
// tile, and Chebyshev interpolation over the whole 1024-point tile converges
// much faster per node than over a quarter, so lines whose centre lies more
// than kFFTier2 (kFFTier3, kFFTier4) points outside the tile are evaluated
// at only 32 (16, 8) Chebyshev points of the whole tile, which lets one
// 64-lane pass take 2 (4, 8) lines.  At the end of the tile each tier's
// interpolant is evaluated at the 64 quarter nodes (a fixed matrix of
// Lagrange basis values) and added to their sums.  In FP32 arithmetic the
// whole chain stays within 2.5e-6 of a line's part at each tier's edge
// (damping 1e-4 to 1e5, Doppler widths of 1 to 100 points).
constexpr int kFFTier2 = 128;
constexpr int kFFTier3 = 384;
constexpr int kFFTier4 = 1536;
constexpr int kFFTileNodes = 32 + 16 + 8;   // nodes of the three whole-tile tiers, in that order
// FP64 far field: the same 64 nodes per tile for lines whose window covers
// the tile, whose |x| < 40 zone misses it (so the four-node fraction holds
// over the whole tile) and whose centre lies more than kFFDist64 points
// outside it.  At that distance the float64 interpolation error stays below
// 1e-12 of the line's part (damping 1e-4 to 1e5, Doppler widths of 1 to 60
// points), under the four-node rule's own 3e-12.
constexpr int kFFDist64 = 384;

// Half-width in fine points of the zone where |x| < R may occur, for a line
// with c1 = ln q / b: |x| >= R implies |d| >= R / (1.02 c1) (|d ln q| <= 0.031).
__host__ __device__ inline int32_t zone_half(double R, double c1) {
  return (int32_t)ceil(R * 1.02 / c1) + 2;
}
// The same from b / ln q = 1 / c1 (a product instead of a quotient).
__host__ __device__ inline int32_t zone_half_b(double R, double b_over_lnq) {
  return (int32_t)ceil(R * 1.02 * b_over_lnq) + 2;
}

// Quadrature constants computed on the host at plan time.
struct QuadConsts {
  float gh2_t2;            // t^2 of the 2-node rule (positive node)
  float gh4_t2[2];         // t_k^2 of the 4-node rule, k = 1, 2
  float gh4_w[2];          // omega_k / pi
  float tr32_ci[2 * kTrap32Half + 1];   // (h/pi) e^{-t^2}, t = k h
  float tr32_ch[2 * kTrap32Half + 1];   // (h/pi) e^{-t^2}, t = (k + 1/2) h
  double gh8_t2[4];        // t_k^2 of the 8-node rule
  double gh8_w[4];         // omega_k / pi
  double gh4_t2d[2];       // t_k^2 of the 4-node rule (FP64)
  double gh4_wd[2];        // omega_k / pi
  double tr64_ci[2 * kTrap64Half + 1];
  double tr64_ch[2 * kTrap64Half + 1];
  float ff_s[kFFNodes];    // Chebyshev points cos((2n + 1) pi / 32)
  float ff_w[kFFNodes];    // their barycentric weights (-1)^n sin((2n + 1) pi / 32)
  float ff_off[64];        // node of lane l, in points after the tile's first point:
                           // Chebyshev point l % 16 of quarter l / 16
  double ff_off64[64];     // the same in FP64
  // whole-tile tiers: node positions (points after the tile's first point)
  // of the 32-, 16- and 8-point Chebyshev sets of the tile, one set after
  // the other, and the Lagrange basis value of each node at each quarter
  // node (ff_V[n][l]: node n at the node of lane l)
  float ff_toff[kFFTileNodes];
  float ff_V[kFFTileNodes][64];
  // FP64 interpolation: the far field at point k of a quarter is
  // sum_n ff_M64[k][n] f_n over its 16 node values f_n (barycentric weights
  // of the Chebyshev points, normalised at each point)
  double ff_M64[kFFQuarter][kFFNodes];
  // T_{2k+1} on interval i: c0 + c1 f + c2 f^2 + c3 f^3, f = s kSerIntervals - i
  alignas(16) float ser[kSerTerms][kSerIntervals][4];
};

// ---- resident line list (sorted by wavelength), structure of arrays --------
struct DevLines {
  int64_t n;
  const double* j0s;     // fractional fine-grid index of the line centre
  const double* amp;     // (pi e^2 / m_e c) g f / (sqrt(pi) nu0)
  const double* e_k;     // E_low / k  [K]
  const double* hc_k;    // h nu0 / k  [K]
  const double* g_rad;   // gamma_rad   / (4 pi nu0)
  const double* g_stark; // gamma_stark / (4 pi nu0)
  const double* g_vdw;   // gamma_vdW   / (4 pi nu0)
  const double* thr;     // cutoff * kappa_c(lambda0)
  const int32_t* sp;     // species
  const int32_t* ss;     // species * n_stages + stage
};

// Per-point state computed on the device.
struct PointState {
  double T;
  double cS;        // n_e (T/1e4)^(1/6)
  double cW;        // N_heavy (T/1e4)^0.3
  double n_e, n_heavy, n_H, rho;
  double pad;
};

// Survivor records, one per kept line and point: the narrow class, then the
// wide one, each in wavelength order (kNarrowHalf).  A
// wave loads the windows of 64 of them at a time (one per lane; for FP32
// records also their (J, czh), from which each lane computes its record's
// row masks), tests them against its tile with one ballot and reads each
// intersecting record with scalar loads.  `czh` holds the half-widths in fine
// points of the zones around the centre where |x + i a| may be below the
// rules' radii (FP32: two 16-bit fields, -32768 for none; FP64: -1 for none).
//
// FP32 far wing: S H = (A v + B) / (v^2 + E), v = u^2 + D, u = sigma x,
//  - two-node Gauss-Hermite pair (a < 1e4), sigma = 1, C1 = S a / sqrt(pi):
//    the pair's fraction C1 (u^2 + a^2 + 1/2) / ((u^2 + a^2 - 1/2)^2 + 2 a^2),
//    so A = B = C1, D = a^2 - 1/2, E = 2 a^2;
//  - Lorentz limit (a >= 1e4, pair correction below 1/(2 a^2)), sigma = 1/a:
//    C1 / (x^2 + a^2) = (C1 / a^2) / (u^2 + 1), so A = C1 / a^2, B = 0,
//    D = 1, E = 0, without overflow at any a.
// In the far wing v >= 224, so writing the denominator as a square plus E
// loses nothing, and a row costs one FMA for v, one for the denominator and
// one for the numerator.  sigma is folded into c1, so the kernel computes u
// directly from the index.
struct alignas(16) Rec32 {
  int32_t J;        // nearest integer of the fractional centre index
  int32_t jlo, jhi; // window, clipped to the grid
  int32_t czh;      // zone half-widths: low 16 bits |x| < 15, high 16 bits |x| < 6 (-32768: none);
                    // the Voigt kernel reads them from the (J, czh) array, this copy completes the record
  float phi;        // fractional centre minus J, in [-1/2, 1/2]
  float c1;         // sigma ln q / b, so u ~= d c1 (1 + d ln q / 2 + ...)
  float A, B, D, E;     // far-wing fraction (above)
  float S;          // line strength
  float y;          // damping parameter a
};
struct alignas(16) Rec64 {
  int32_t J, jlo, jhi;
  int32_t czh;      // half-width of the zone where |x| < 8 may occur (-1: none)
  int32_t z40;      // the same for |x| < 40 (the kernel reads it from the (J, z40) array)
  int32_t li;       // sorted line index (stage checks)
  int32_t pad0, pad1;
  double phi, S, y, c1;
};

struct Batch {
  // all pointers are into the workspace; strides per point
  int32_t n_points;
  const double* T;      // [B]
  const double* log10P; // [B]
  const double* vt_kms; // [B]
  const double* abundance;  // [S]
  PointState* state;    // [B]
  double* pop;          // [B][S*K]
  double* bT;           // [B][S][2]: b and 1/b
  ulonglong2* keep;     // [L]          per line, bit p of x: kept at point p; of y: kept in the wide class
  int2* wline;          // [B][L]       survivors' windows (j_lo, j_hi) by line, from the selection
  int32_t* blk;         // [B][2][nblk] counts per class, then offsets within the class
  int32_t* nsurv;       // [B]         survivors (both classes)
  int32_t* nsurv_n;     // [B]         narrow survivors (the first nsurv_n records)
  int32_t* hmax;        // [B]         max half-window of the narrow class, in fine points
  int32_t* hmax_w;      // [B]         max half-window of the wide class
  unsigned long long* nsamp;  // [B]
  int32_t* nit;         // [B]         ionisation-equilibrium steps (0: fixed P_e; < 0: not converged)
  void* rec;            // [B][L] Rec32 or Rec64
  int2* win;            // [B][L] (jlo, jhi) of each record, scanned by the Voigt kernels
  int2* wz;             // [B][L] (J, czh) of each FP32 record or (J, z40) of each FP64 one, read
                        //        with its window
  void* kappa;          // [B][N] float or double
  int64_t rec_stride;   // = L
  int64_t kappa_stride; // = N
};

struct Params {
  int32_t n_species, n_stages;
  const double* mass_amu;  // device [S]
  const double* chi_ev;    // device [S][K-1]
  const double* part_fn;   // device [S][K]
  double pe_over_p;
  double cutoff, cap;
  double lnq;              // ln(1 + 1/R), FP64
  double lambda_first_nm;
  double kc_ref, kc_lref, kc_power;   // kappa_c = kc_ref (lambda / kc_lref)^kc_power
  int64_t N;
  int32_t n_bins, n_steps;
  const int64_t* edges;    // device [n_bins+1]
  const double* Fcum;      // device [n_steps+1] cumulative fractions, F[0]=0, F[n]=1
  const void* floor;       // device [N], float (mixed) or double: cutoff * kappa_c(lambda_j)
  int32_t mean;            // 0 geometric, 1 arithmetic
  int32_t precision;       // 0 fp64, 1 mixed
  int32_t output;          // 0 ODF table, 1 fine-grid opacity
  int32_t electrons;       // 0 fixed P_e / P, 1 ionisation equilibrium
  int32_t ne_max_iter;     // Newton steps allowed to the ionisation equilibrium
};

// ---- launchers (defined in the .hip files) ---------------------------------
hipError_t launch_prep_lines(hipStream_t st, int64_t n, const double* lam_nm, const double* log_gf,
                             const double* e_ev, const double* lg_rad, const double* lg_stark,
                             const double* lg_vdw, const int32_t* species, const int32_t* stage,
                             int32_t n_stages, double lambda_first_nm, double lnq, double cutoff,
                             double kc_ref, double kc_lref, double kc_pow,
                             double* j0s, double* amp, double* e_k, double* hc_k, double* g_rad,
                             double* g_stark, double* g_vdw, double* thr, int32_t* ss);
hipError_t launch_point_state(hipStream_t st, const Params& P, const Batch& B);
hipError_t launch_select(hipStream_t st, const Params& P, const DevLines& L, const Batch& B);
hipError_t launch_scan(hipStream_t st, const Params& P, const DevLines& L, const Batch& B);
hipError_t launch_emit(hipStream_t st, const Params& P, const DevLines& L, const Batch& B, int rec64);
hipError_t launch_voigt(hipStream_t st, const Params& P, const Batch& B, const QuadConsts* Q);
// The opacity floor cutoff * kappa_c(lambda_j) at every fine point, in the
// path's type, into P.floor (once per plan).
hipError_t launch_floor(hipStream_t st, const Params& P, void* floor);
// Floored fine-grid opacity of n_points grids (kappa rows kappa_stride apart)
// into out [n_points][N].
hipError_t launch_fine(hipStream_t st, const Params& P, const void* kappa, int64_t kappa_stride,
                       int32_t n_points, void* out);
// Bins grouped by padded size (power of two) so each ODF launch reserves only
// the LDS its largest bin needs.  bins: device list of bin indices, class c at
// [offset[c], offset[c] + count[c]).
constexpr int kMaxOdfClasses = 32;
struct OdfClasses {
  int n_classes;
  int npow2[kMaxOdfClasses];
  int offset[kMaxOdfClasses];
  int count[kMaxOdfClasses];
  const int32_t* bins;
};
hipError_t launch_odf(hipStream_t st, const Params& P, const void* kappa, int64_t kappa_stride,
                      int32_t n_points, void* out, const OdfClasses& C, void* gscratch,
                      const int64_t* goff, int64_t gscratch_stride);
// largest bin (in points) that the ODF kernel sorts in LDS
inline int odf_lds_cap(int precision) { return (128 * 1024) / (precision == 1 ? 4 : 8); }

inline int64_t n_line_blocks(int64_t n) { return (n + kLineBlock - 1) / kLineBlock; }

}  // namespace odf

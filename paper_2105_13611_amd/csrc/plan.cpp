// Plan construction, validation, workspace carving, the blocking compute
// path and the per-stage entry points of the ODF engine (C ABI, include/odf.h).
#include "plan.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "loop.h"

namespace odf {

thread_local std::string g_err;

std::string g_last_error_copy() { return g_err; }
void g_last_error_clear() { g_err.clear(); }

void set_error(const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
}

namespace {

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) {                                                            \
      set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), __FILE__, __LINE__); \
      return ODF_E_DEVICE;                                                             \
    }                                                                                  \
  } while (0)

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int64_t grid_points(double lf, double ll, double R) {
  if (!finite_pos(lf) || !finite_pos(ll) || !finite_pos(R) || ll < lf) return -1;
  // N = floor(ln(ll/lf) / ln(1 + 1/R)) + 1, taken in long double
  const long double v = std::log((long double)ll / (long double)lf) / std::log1p(1.0L / (long double)R);
  if (v > 2.0e9L) return -1;
  return (int64_t)std::floor(v) + 1;
}

template <typename T>
odf_status dev_alloc(odf_plan_s* p, T** ptr, int64_t count) {
  void* d = nullptr;
  if (count > 0) {
    hipError_t e = hipMalloc(&d, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
      set_error("hipMalloc of %lld bytes failed: %s", (long long)(count * sizeof(T)),
                hipGetErrorString(e));
      return ODF_E_DEVICE;
    }
    p->owned.push_back(d);
  }
  *ptr = static_cast<T*>(d);
  return ODF_OK;
}

void free_owned(odf_plan_s* p) {
  for (void* d : p->owned) (void)hipFree(d);
  p->owned.clear();
}

// Streams and events of the odf_compute pipeline (null handles skipped).
void release_streams(odf_plan_s* p) {
  if (p->prep_stream) (void)hipStreamDestroy(p->prep_stream);
  for (hipStream_t& st : p->sum_stream)
    if (st) (void)hipStreamDestroy(st);
  for (hipEvent_t& e : p->ev_join)
    if (e) (void)hipEventDestroy(e);
  for (int k = 0; k < kPipeSlots; ++k) {
    if (p->ev_prep[k]) (void)hipEventDestroy(p->ev_prep[k]);
    if (p->ev_free[k]) (void)hipEventDestroy(p->ev_free[k]);
  }
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  p->prep_stream = nullptr;
  p->sum_stream[0] = p->sum_stream[1] = nullptr;
  p->ev_fork = nullptr;
  for (hipEvent_t& e : p->ev_join) e = nullptr;
  for (int k = 0; k < kPipeSlots; ++k) p->ev_prep[k] = p->ev_free[k] = nullptr;
}

odf_status validate_layout(const odf_layout* L, int64_t* N_out) {
  if (!L) { set_error("layout is NULL"); return ODF_E_INVALID; }
  const int64_t N = grid_points(L->lambda_first_nm, L->lambda_last_nm, L->resolving_power);
  if (N < 1) {
    set_error("layout: need 0 < lambda_first_nm <= lambda_last_nm and resolving_power > 0 (grid of at most 2e9 points)");
    return ODF_E_INVALID;
  }
  if (L->n_bins < 1 || !L->bin_edges) { set_error("layout: n_bins must be >= 1 with bin_edges"); return ODF_E_INVALID; }
  if (L->bin_edges[0] < 0 || L->bin_edges[L->n_bins] > N) {
    set_error("layout: bin_edges must lie within [0, N=%lld]", (long long)N);
    return ODF_E_INVALID;
  }
  for (int b = 0; b < L->n_bins; ++b) {
    const int64_t w = L->bin_edges[b + 1] - L->bin_edges[b];
    if (w <= 0) { set_error("layout: bin_edges not strictly increasing at bin %d", b); return ODF_E_INVALID; }
    if (w > (1 << 20)) { set_error("layout: bin %d has %lld points (max 1048576)", b, (long long)w); return ODF_E_INVALID; }
  }
  if (L->n_steps < 1 || !L->step_frac) { set_error("layout: n_steps must be >= 1 with step_frac"); return ODF_E_INVALID; }
  double s = 0.0;
  for (int k = 0; k < L->n_steps; ++k) {
    if (!finite_pos(L->step_frac[k])) { set_error("layout: step_frac[%d] must be finite and > 0", k); return ODF_E_INVALID; }
    s += L->step_frac[k];
  }
  if (std::fabs(s - 1.0) > 1e-9) { set_error("layout: step_frac sums to %.17g, not 1", s); return ODF_E_INVALID; }
  *N_out = N;
  return ODF_OK;
}

odf_status validate_lines(const odf_lines* l, const odf_species* sp) {
  if (!l) { set_error("lines is NULL"); return ODF_E_INVALID; }
  if (!sp) { set_error("species is NULL"); return ODF_E_INVALID; }
  if (sp->n_species < 1 || sp->n_stages < 1 || sp->n_stages > 8) {
    set_error("species: need n_species >= 1 and 1 <= n_stages <= 8");
    return ODF_E_INVALID;
  }
  if (!sp->mass_amu || !sp->part_fn || (sp->n_stages > 1 && !sp->chi_ev)) {
    set_error("species: NULL array");
    return ODF_E_INVALID;
  }
  for (int s = 0; s < sp->n_species; ++s) {
    if (!finite_pos(sp->mass_amu[s])) { set_error("species: mass_amu[%d] must be > 0", s); return ODF_E_INVALID; }
    for (int k = 0; k < sp->n_stages; ++k)
      if (!finite_pos(sp->part_fn[s * sp->n_stages + k])) {
        set_error("species: part_fn[%d][%d] must be > 0", s, k);
        return ODF_E_INVALID;
      }
    for (int k = 0; k + 1 < sp->n_stages; ++k)
      if (!std::isfinite(sp->chi_ev[s * (sp->n_stages - 1) + k])) {
        set_error("species: chi_ev[%d][%d] not finite", s, k);
        return ODF_E_INVALID;
      }
  }
  if (l->n_lines < 0 || l->n_lines > (int64_t)INT32_MAX - 1) {
    set_error("lines: n_lines must be in [0, 2^31-2]");
    return ODF_E_INVALID;
  }
  if (l->n_lines > 0 && (!l->lambda_nm || !l->log_gf || !l->e_low_ev || !l->species || !l->stage ||
                         !l->log_g_rad || !l->log_g_stark || !l->log_g_vdw)) {
    set_error("lines: NULL array");
    return ODF_E_INVALID;
  }
  for (int64_t i = 0; i < l->n_lines; ++i) {
    if (!finite_pos(l->lambda_nm[i])) { set_error("lines: lambda_nm[%lld] must be finite and > 0", (long long)i); return ODF_E_INVALID; }
    if (!std::isfinite(l->log_gf[i]) || !std::isfinite(l->e_low_ev[i]) || !std::isfinite(l->log_g_rad[i]) ||
        !std::isfinite(l->log_g_stark[i]) || !std::isfinite(l->log_g_vdw[i])) {
      set_error("lines: non-finite value in line %lld", (long long)i);
      return ODF_E_INVALID;
    }
    if (l->species[i] < 0 || l->species[i] >= sp->n_species) {
      set_error("lines: species[%lld] = %d out of range [0, %d)", (long long)i, l->species[i], sp->n_species);
      return ODF_E_INVALID;
    }
    if (l->stage[i] < 0 || l->stage[i] >= sp->n_stages) {
      set_error("lines: stage[%lld] = %d out of range [0, %d)", (long long)i, l->stage[i], sp->n_stages);
      return ODF_E_INVALID;
    }
  }
  return ODF_OK;
}

odf_status validate_options(const odf_options* o) {
  if (!o) { set_error("options is NULL"); return ODF_E_INVALID; }
  if (o->precision != ODF_PREC_FP64 && o->precision != ODF_PREC_MIXED) { set_error("options: bad precision"); return ODF_E_INVALID; }
  if (o->mean != ODF_MEAN_GEOMETRIC && o->mean != ODF_MEAN_ARITHMETIC) { set_error("options: bad mean"); return ODF_E_INVALID; }
  if (!finite_pos(o->cutoff)) { set_error("options: cutoff must be > 0"); return ODF_E_INVALID; }
  if (!finite_pos(o->window_cap_doppler) || o->window_cap_doppler > 2000.0) {
    set_error("options: window_cap_doppler must be in (0, 2000]");
    return ODF_E_INVALID;
  }
  if (o->output != ODF_OUT_TABLE && o->output != ODF_OUT_FINE) { set_error("options: bad output"); return ODF_E_INVALID; }
  if (o->electrons != ODF_NE_FIXED && o->electrons != ODF_NE_EQUILIBRIUM) { set_error("options: bad electrons"); return ODF_E_INVALID; }
  if (o->electrons == ODF_NE_FIXED && !(o->pe_over_p > 0.0 && o->pe_over_p < 1.0)) {
    set_error("options: pe_over_p must be in (0, 1)");
    return ODF_E_INVALID;
  }
  if (!finite_pos(o->kappa_c_ref) || !finite_pos(o->lambda_c_ref_nm) || !std::isfinite(o->kappa_c_power)) {
    set_error("options: continuum parameters must be finite, reference values > 0");
    return ODF_E_INVALID;
  }
  if (!o->workspace || o->workspace_bytes <= 0) { set_error("options: workspace and workspace_bytes required"); return ODF_E_INVALID; }
  if (o->max_batch_points < 0 || o->loop_streams < 0 || o->loop_streams > 8) {
    set_error("options: max_batch_points >= 0 and loop_streams in [0, 8]");
    return ODF_E_INVALID;
  }
  return ODF_OK;
}

}  // namespace

// Offsets of one batch slot holding `pts` points.
SlotLayout make_slot(const odf_plan_s* p, int32_t pts) {
  SlotLayout s{};
  const int64_t L = p->n_lines, S = p->n_species, K = p->n_stages;
  const int64_t nblk = n_line_blocks(L);
  const bool mixed = p->opts.precision == ODF_PREC_MIXED;
  int64_t o = 0;
  auto take = [&](int64_t bytes) { const int64_t at = o; o += align_up(bytes); return at; };
  s.off_T = take(8 * pts);
  s.off_logP = take(8 * pts);
  s.off_vt = take(8 * pts);
  s.off_abund = take(8 * S);
  s.off_state = take((int64_t)sizeof(PointState) * pts);
  s.off_pop = take(8 * S * K * pts);
  s.off_bT = take(16 * S * pts);   // (b, 1/b) per species
  s.off_keep = take(16 * std::max<int64_t>(L, 1));
  s.off_wline = take((int64_t)sizeof(int2) * std::max<int64_t>(L, 1) * pts);
  s.off_blk = take(4 * 2 * std::max<int64_t>(nblk, 1) * pts);
  s.off_nsurv = take(4 * pts);
  s.off_nsurv_n = take(4 * pts);
  s.off_hmax = take(4 * pts);
  s.off_hmax_w = take(4 * pts);
  s.off_nsamp = take(8 * pts);
  s.off_nit = take(4 * pts);
  s.off_rec = take((mixed ? (int64_t)sizeof(Rec32) : (int64_t)sizeof(Rec64)) * std::max<int64_t>(L, 1) * pts);
  s.off_win = take((int64_t)sizeof(int2) * std::max<int64_t>(L, 1) * pts);
  s.off_wz = take((int64_t)sizeof(int2) * std::max<int64_t>(L, 1) * pts);
  s.off_kappa = take((mixed ? 4 : 8) * p->N * pts);
  s.off_gscr = take((mixed ? 4 : 8) * std::max<int64_t>(p->gscr_elems, 1) * pts);
  s.bytes = o;
  s.points = pts;
  return s;
}

Batch make_batch(const odf_plan_s* p, const SlotLayout& s, char* base, int32_t n_points) {
  Batch B{};
  B.n_points = n_points;
  B.T = reinterpret_cast<const double*>(base + s.off_T);
  B.log10P = reinterpret_cast<const double*>(base + s.off_logP);
  B.vt_kms = reinterpret_cast<const double*>(base + s.off_vt);
  B.abundance = reinterpret_cast<const double*>(base + s.off_abund);
  B.state = reinterpret_cast<PointState*>(base + s.off_state);
  B.pop = reinterpret_cast<double*>(base + s.off_pop);
  B.bT = reinterpret_cast<double*>(base + s.off_bT);
  B.keep = reinterpret_cast<ulonglong2*>(base + s.off_keep);
  B.wline = reinterpret_cast<int2*>(base + s.off_wline);
  B.blk = reinterpret_cast<int32_t*>(base + s.off_blk);
  B.nsurv = reinterpret_cast<int32_t*>(base + s.off_nsurv);
  B.nsurv_n = reinterpret_cast<int32_t*>(base + s.off_nsurv_n);
  B.hmax = reinterpret_cast<int32_t*>(base + s.off_hmax);
  B.hmax_w = reinterpret_cast<int32_t*>(base + s.off_hmax_w);
  B.nsamp = reinterpret_cast<unsigned long long*>(base + s.off_nsamp);
  B.nit = reinterpret_cast<int32_t*>(base + s.off_nit);
  B.rec = base + s.off_rec;
  B.win = reinterpret_cast<int2*>(base + s.off_win);
  B.wz = reinterpret_cast<int2*>(base + s.off_wz);
  B.kappa = base + s.off_kappa;
  B.rec_stride = std::max<int64_t>(p->n_lines, 1);
  B.kappa_stride = p->N;
  return B;
}

// Enqueue the whole per-point chain for the points already staged in `B`:
// state -> selection -> scan -> survivor emission -> Voigt -> ODF.
namespace {

// Records an event pair around one launch when timing is on.
struct TimedLaunch {
  StageTimer* t;
  hipStream_t st;
  size_t pair = 0;
  TimedLaunch(StageTimer* timer, hipStream_t s, int stage) : t(timer), st(s) {
    if (!t) return;
    if (2 * (t->used + 1) > t->pool.size()) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { t = nullptr; return; }
      t->pool.push_back(a);
      t->pool.push_back(b);
      t->stage_of_pair.push_back(0);
    }
    pair = t->used++;
    t->stage_of_pair[pair] = stage;
    (void)hipEventRecord(t->pool[2 * pair], st);
  }
  ~TimedLaunch() {
    if (t) (void)hipEventRecord(t->pool[2 * pair + 1], st);
  }
};

}  // namespace

odf_status enqueue_prep(odf_plan_s* p, const Batch& B, hipStream_t st, StageTimer* timer) {
  { TimedLaunch tl(timer, st, 0); HIP_TRY(launch_point_state(st, p->params, B)); }
  { TimedLaunch tl(timer, st, 1); HIP_TRY(launch_select(st, p->params, p->lines, B)); }
  { TimedLaunch tl(timer, st, 2); HIP_TRY(launch_scan(st, p->params, p->lines, B)); }
  { TimedLaunch tl(timer, st, 3); HIP_TRY(launch_emit(st, p->params, p->lines, B, p->opts.precision == ODF_PREC_FP64)); }
  return ODF_OK;
}

odf_status enqueue_sum(odf_plan_s* p, const Batch& B, char* slot_base, const SlotLayout& s,
                       void* out, hipStream_t st, StageTimer* timer) {
  { TimedLaunch tl(timer, st, 4); HIP_TRY(launch_voigt(st, p->params, B, p->d_quad)); }
  if (out) {
    TimedLaunch tl(timer, st, 5);
    if (p->params.output == 1)
      HIP_TRY(launch_fine(st, p->params, B.kappa, B.kappa_stride, B.n_points, out));
    else
      HIP_TRY(launch_odf(st, p->params, B.kappa, B.kappa_stride, B.n_points, out, p->odf_classes,
                         slot_base + s.off_gscr, p->d_goff, p->gscr_elems));
  }
  return ODF_OK;
}

size_t out_point_bytes(const odf_plan_s* p) {
  const size_t osz = p->opts.precision == ODF_PREC_MIXED ? 4 : 8;
  const size_t n = p->opts.output == ODF_OUT_FINE ? (size_t)p->N : (size_t)p->n_bins * p->n_steps;
  return n * osz;
}

odf_status enqueue_batch(odf_plan_s* p, const Batch& B, char* slot_base, const SlotLayout& s,
                         void* out, hipStream_t st, StageTimer* timer) {
  const odf_status e = enqueue_prep(p, B, st, timer);
  if (e != ODF_OK) return e;
  return enqueue_sum(p, B, slot_base, s, out, st, timer);
}

// After the streams have drained: add the recorded pairs to the totals.
// Launches on different streams may overlap, so besides the summed
// durations each stage gets the length of the union of its launch intervals
// (times taken relative to the first recorded event).
void collect_timer(StageTimer& t) {
  std::vector<std::pair<float, float>> iv[kStages];
  for (size_t i = 0; i < t.used; ++i) {
    float ms = 0.0f, t0 = 0.0f, t1 = 0.0f;
    if (hipEventElapsedTime(&ms, t.pool[2 * i], t.pool[2 * i + 1]) != hipSuccess) continue;
    const int k = t.stage_of_pair[i];
    t.ms[k] += ms;
    t.launches[k] += 1;
    if (hipEventElapsedTime(&t0, t.pool[0], t.pool[2 * i]) == hipSuccess &&
        hipEventElapsedTime(&t1, t.pool[0], t.pool[2 * i + 1]) == hipSuccess)
      iv[k].emplace_back(t0, t1);
  }
  for (int k = 0; k < kStages; ++k) {
    std::sort(iv[k].begin(), iv[k].end());
    double total = 0.0, a = 0.0, b = 0.0;
    bool open = false;
    for (const auto& x : iv[k]) {
      if (open && x.first <= b) {
        b = std::max(b, (double)x.second);
        continue;
      }
      if (open) total += b - a;
      a = x.first;
      b = x.second;
      open = true;
    }
    if (open) total += b - a;
    t.busy_ms[k] += total;
  }
  t.used = 0;
}

odf_status validate_request(const odf_plan_s* p, const odf_request* r, bool need_out) {
  if (!r) { set_error("request is NULL"); return ODF_E_INVALID; }
  if (r->n_points < 0) { set_error("request: n_points < 0"); return ODF_E_INVALID; }
  if (!r->abundance) { set_error("request: abundance is NULL"); return ODF_E_INVALID; }
  for (int s = 0; s < p->n_species; ++s)
    if (!finite_pos(r->abundance[s])) { set_error("request: abundance[%d] must be finite and > 0", s); return ODF_E_INVALID; }
  if (r->n_points > 0) {
    if (!r->T_K || !r->log10_P_cgs || !r->vturb_kms) { set_error("request: NULL point array"); return ODF_E_INVALID; }
    if (need_out && !r->out) { set_error("request: out is NULL"); return ODF_E_INVALID; }
  }
  for (int i = 0; i < r->n_points; ++i) {
    if (!finite_pos(r->T_K[i]) || r->T_K[i] > 1e9) { set_error("request: T_K[%d] must be finite, > 0 and <= 1e9", i); return ODF_E_INVALID; }
    if (!std::isfinite(r->log10_P_cgs[i]) || std::fabs(r->log10_P_cgs[i]) > 30.0) {
      set_error("request: log10_P_cgs[%d] must be finite with |value| <= 30", i);
      return ODF_E_INVALID;
    }
    if (!std::isfinite(r->vturb_kms[i]) || r->vturb_kms[i] < 0.0 || r->vturb_kms[i] > 1000.0) {
      set_error("request: vturb_kms[%d] must be in [0, 1000]", i);
      return ODF_E_INVALID;
    }
  }
  return ODF_OK;
}

}  // namespace odf

using namespace odf;

extern "C" {

const char* odf_last_error(void) { return g_err.c_str(); }

int64_t odf_grid_points(const odf_layout* layout) {
  if (!layout) return -1;
  return grid_points(layout->lambda_first_nm, layout->lambda_last_nm, layout->resolving_power);
}

odf_status odf_plan(const odf_lines* lines, const odf_species* species, const odf_layout* layout,
                    const odf_options* opts, odf_plan_t** out) {
  g_err.clear();
  if (!out) { set_error("out is NULL"); return ODF_E_INVALID; }
  *out = nullptr;
  int64_t N = 0;
  odf_status st;
  if ((st = validate_options(opts)) != ODF_OK) return st;
  if ((st = validate_layout(layout, &N)) != ODF_OK) return st;
  if ((st = validate_lines(lines, species)) != ODF_OK) return st;
  if (N > (int64_t)INT32_MAX - 2 * kWGPoints) { set_error("layout: grid too large"); return ODF_E_INVALID; }

  std::unique_ptr<odf_plan_s> p(new odf_plan_s());
  p->opts = *opts;
  HIP_TRY(hipGetDevice(&p->device));
  // the allocation-free reduction's static scratch: its address on this
  // device, resolved here once so that odf_reduce_noalloc needs no set-up
  if (!noalloc_scratch(p->device)) return ODF_E_DEVICE;
  if (p->opts.loop_streams == 0) p->opts.loop_streams = 2;
  p->n_species = species->n_species;
  p->n_stages = species->n_stages;
  p->n_lines = lines->n_lines;
  p->N = N;
  p->n_bins = layout->n_bins;
  p->n_steps = layout->n_steps;
  p->lambda_first_nm = layout->lambda_first_nm;
  p->lambda_last_nm = layout->lambda_last_nm;
  p->resolving_power = layout->resolving_power;
  p->lnq = std::log1p(1.0 / layout->resolving_power);
  p->edges.assign(layout->bin_edges, layout->bin_edges + layout->n_bins + 1);
  p->Fcum.assign(layout->n_steps + 1, 0.0);
  for (int k = 0; k < layout->n_steps; ++k) p->Fcum[k + 1] = p->Fcum[k] + layout->step_frac[k];
  const double Ftot = p->Fcum[layout->n_steps];
  for (auto& f : p->Fcum) f = f / Ftot;
  p->max_bin = 0;
  for (int b = 0; b < p->n_bins; ++b)
    p->max_bin = std::max<int32_t>(p->max_bin, (int32_t)(p->edges[b + 1] - p->edges[b]));

  // ODF global scratch for bins too large for LDS
  const int cap = odf_lds_cap(p->opts.precision == ODF_PREC_MIXED ? 1 : 0);
  std::vector<int64_t> goff(p->n_bins, 0);
  int64_t g = 0;
  for (int b = 0; b < p->n_bins; ++b) {
    int64_t n = p->edges[b + 1] - p->edges[b], pw = 1;
    while (pw < n) pw <<= 1;
    if (pw > cap) { goff[b] = g; g += pw; }
  }
  p->gscr_elems = g;

  // sort lines by wavelength (stable: equal wavelengths keep input order)
  const int64_t L = lines->n_lines;
  p->orig.resize(L);
  std::iota(p->orig.begin(), p->orig.end(), 0);
  std::stable_sort(p->orig.begin(), p->orig.end(), [&](int64_t a, int64_t b) {
    return lines->lambda_nm[a] < lines->lambda_nm[b];
  });
  hipStream_t s0 = static_cast<hipStream_t>(p->opts.stream);
  {
    std::vector<double> tmp(L);
    std::vector<int32_t> tmpi(L);
    double *r_lam, *r_gf, *r_e, *r_gr, *r_gs, *r_gw;
    int32_t *r_sp, *r_st;
    odf_plan_s* pp = p.get();
    if ((st = dev_alloc(pp, &r_lam, L)) || (st = dev_alloc(pp, &r_gf, L)) || (st = dev_alloc(pp, &r_e, L)) ||
        (st = dev_alloc(pp, &r_gr, L)) || (st = dev_alloc(pp, &r_gs, L)) || (st = dev_alloc(pp, &r_gw, L)) ||
        (st = dev_alloc(pp, &r_st, L))) {
      free_owned(pp);
      return st;
    }
    double *j0s, *amp, *e_k, *hc_k, *g_rad, *g_stark, *g_vdw, *thr;
    int32_t *sp, *ss;
    if ((st = dev_alloc(pp, &j0s, L)) || (st = dev_alloc(pp, &amp, L)) || (st = dev_alloc(pp, &e_k, L)) ||
        (st = dev_alloc(pp, &hc_k, L)) || (st = dev_alloc(pp, &g_rad, L)) ||
        (st = dev_alloc(pp, &g_stark, L)) || (st = dev_alloc(pp, &g_vdw, L)) ||
        (st = dev_alloc(pp, &thr, L)) || (st = dev_alloc(pp, &sp, L)) || (st = dev_alloc(pp, &ss, L))) {
      free_owned(pp);
      return st;
    }
    r_sp = sp;  // species array is kept resident as is
    auto up = [&](double* d, const double* src) -> hipError_t {
      for (int64_t i = 0; i < L; ++i) tmp[i] = src[p->orig[i]];
      return hipMemcpy(d, tmp.data(), L * sizeof(double), hipMemcpyHostToDevice);
    };
    auto upi = [&](int32_t* d, const int32_t* src) -> hipError_t {
      for (int64_t i = 0; i < L; ++i) tmpi[i] = src[p->orig[i]];
      return hipMemcpy(d, tmpi.data(), L * sizeof(int32_t), hipMemcpyHostToDevice);
    };
    hipError_t e = hipSuccess;
    if (L > 0) {
      if ((e = up(r_lam, lines->lambda_nm)) != hipSuccess || (e = up(r_gf, lines->log_gf)) != hipSuccess ||
          (e = up(r_e, lines->e_low_ev)) != hipSuccess || (e = up(r_gr, lines->log_g_rad)) != hipSuccess ||
          (e = up(r_gs, lines->log_g_stark)) != hipSuccess || (e = up(r_gw, lines->log_g_vdw)) != hipSuccess ||
          (e = upi(r_sp, lines->species)) != hipSuccess || (e = upi(r_st, lines->stage)) != hipSuccess) {
        set_error("line upload failed: %s", hipGetErrorString(e));
        free_owned(pp);
        return ODF_E_DEVICE;
      }
      e = launch_prep_lines(s0, L, r_lam, r_gf, r_e, r_gr, r_gs, r_gw, r_sp, r_st, p->n_stages,
                            p->lambda_first_nm, p->lnq, p->opts.cutoff, p->opts.kappa_c_ref,
                            p->opts.lambda_c_ref_nm, p->opts.kappa_c_power, j0s, amp, e_k, hc_k,
                            g_rad, g_stark, g_vdw, thr, ss);
      if (e == hipSuccess) e = hipStreamSynchronize(s0);
      if (e != hipSuccess) {
        set_error("line preparation failed: %s", hipGetErrorString(e));
        free_owned(pp);
        return ODF_E_DEVICE;
      }
    }
    // the raw wavelength-ordered inputs are no longer needed
    for (void* d : {(void*)r_lam, (void*)r_gf, (void*)r_e, (void*)r_gr, (void*)r_gs, (void*)r_gw,
                     (void*)r_st}) {
      if (!d) continue;
      (void)hipFree(d);
      pp->owned.erase(std::remove(pp->owned.begin(), pp->owned.end(), d), pp->owned.end());
    }
    p->lines = DevLines{L, j0s, amp, e_k, hc_k, g_rad, g_stark, g_vdw, thr, sp, ss};
  }

  // species, layout and parameters
  {
    odf_plan_s* pp = p.get();
    double *mass, *chi, *part, *Fc;
    int64_t* edges;
    const int S = p->n_species, K = p->n_stages;
    // bins grouped by padded size for the ODF launches
    std::vector<int32_t> order;
    {
      std::map<int, std::vector<int32_t>> cls;
      for (int b = 0; b < p->n_bins; ++b) {
        int64_t n = p->edges[b + 1] - p->edges[b], pw = 1;
        while (pw < n) pw <<= 1;
        cls[(int)pw].push_back(b);
      }
      if ((int)cls.size() > kMaxOdfClasses) {
        set_error("layout: too many distinct bin sizes");
        free_owned(pp);
        return ODF_E_INVALID;
      }
      OdfClasses& C = pp->odf_classes;
      C.n_classes = 0;
      for (auto& kv : cls) {
        C.npow2[C.n_classes] = kv.first;
        C.offset[C.n_classes] = (int)order.size();
        C.count[C.n_classes] = (int)kv.second.size();
        order.insert(order.end(), kv.second.begin(), kv.second.end());
        ++C.n_classes;
      }
    }
    int32_t* binlist = nullptr;
    if ((st = dev_alloc(pp, &binlist, std::max<int64_t>(p->n_bins, 1)))) { free_owned(pp); return st; }
    pp->odf_classes.bins = binlist;
    if (hipMemcpy(binlist, order.data(), order.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("bin list upload failed");
      free_owned(pp);
      return ODF_E_DEVICE;
    }
    if ((st = dev_alloc(pp, &mass, S)) || (st = dev_alloc(pp, &chi, std::max(S * (K - 1), 1))) ||
        (st = dev_alloc(pp, &part, S * K)) || (st = dev_alloc(pp, &Fc, p->n_steps + 1)) ||
        (st = dev_alloc(pp, &edges, p->n_bins + 1)) ||
        (st = dev_alloc(pp, &pp->d_goff, std::max(p->n_bins, 1)))) {
      free_owned(pp);
      return st;
    }
    hipError_t e = hipSuccess;
    if ((e = hipMemcpy(mass, species->mass_amu, S * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (K > 1 && (e = hipMemcpy(chi, species->chi_ev, S * (K - 1) * 8, hipMemcpyHostToDevice)) != hipSuccess) ||
        (e = hipMemcpy(part, species->part_fn, S * K * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(Fc, p->Fcum.data(), (p->n_steps + 1) * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(edges, p->edges.data(), (p->n_bins + 1) * 8, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(pp->d_goff, goff.data(), p->n_bins * 8, hipMemcpyHostToDevice)) != hipSuccess) {
      set_error("parameter upload failed: %s", hipGetErrorString(e));
      free_owned(pp);
      return ODF_E_DEVICE;
    }
    Params& P = p->params;
    P.n_species = S;
    P.n_stages = K;
    P.mass_amu = mass;
    P.chi_ev = chi;
    P.part_fn = part;
    P.pe_over_p = p->opts.pe_over_p;
    P.cutoff = p->opts.cutoff;
    P.cap = p->opts.window_cap_doppler;
    P.lnq = p->lnq;
    P.lambda_first_nm = p->lambda_first_nm;
    P.kc_ref = p->opts.kappa_c_ref;
    P.kc_lref = p->opts.lambda_c_ref_nm;
    P.kc_power = p->opts.kappa_c_power;
    P.N = p->N;
    P.n_bins = p->n_bins;
    P.n_steps = p->n_steps;
    P.edges = edges;
    P.Fcum = Fc;
    P.mean = p->opts.mean == ODF_MEAN_ARITHMETIC ? 1 : 0;
    P.precision = p->opts.precision == ODF_PREC_MIXED ? 1 : 0;
    P.output = p->opts.output == ODF_OUT_FINE ? 1 : 0;
    P.electrons = p->opts.electrons == ODF_NE_EQUILIBRIUM ? 1 : 0;
    P.ne_max_iter = kNeMaxSteps;
    // the opacity floor per fine point, tabulated once
    void* fl = nullptr;
    if (P.precision == 1) {
      float* f = nullptr;
      st = dev_alloc(pp, &f, std::max<int64_t>(p->N, 1));
      fl = f;
    } else {
      double* f = nullptr;
      st = dev_alloc(pp, &f, std::max<int64_t>(p->N, 1));
      fl = f;
    }
    if (st != ODF_OK) { free_owned(pp); return st; }
    P.floor = fl;
    if ((e = launch_floor(s0, P, fl)) != hipSuccess || (e = hipStreamSynchronize(s0)) != hipSuccess) {
      set_error("opacity floor tabulation failed: %s", hipGetErrorString(e));
      free_owned(pp);
      return ODF_E_DEVICE;
    }
  }
  p->quad = make_quad_consts();
  {
    odf_plan_s* pp = p.get();
    if ((st = dev_alloc(pp, &pp->d_quad, 1)) != ODF_OK) { free_owned(pp); return st; }
    hipError_t e = hipMemcpy(pp->d_quad, &pp->quad, sizeof(QuadConsts), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      set_error("quadrature upload failed: %s", hipGetErrorString(e));
      free_owned(pp);
      return ODF_E_DEVICE;
    }
  }

  // workspace: points per odf_compute batch
  const SlotLayout one = make_slot(p.get(), 1);
  const SlotLayout two = make_slot(p.get(), 2);
  p->per_point_bytes = two.bytes - one.bytes;
  p->fixed_bytes = one.bytes - p->per_point_bytes;
  if (p->opts.workspace_bytes < one.bytes) {
    set_error("workspace of %lld bytes is smaller than one point needs (%lld bytes)",
              (long long)p->opts.workspace_bytes, (long long)one.bytes);
    free_owned(p.get());
    return ODF_E_NOMEM;
  }
  int32_t pts = (int32_t)std::min<int64_t>(
      (p->opts.workspace_bytes - p->fixed_bytes) / std::max<int64_t>(p->per_point_bytes, 1), kMaxBatch);
  if (p->opts.max_batch_points > 0) pts = std::min(pts, p->opts.max_batch_points);
  while (pts > 1 && make_slot(p.get(), pts).bytes > p->opts.workspace_bytes) --pts;
  p->compute_points = std::max(pts, 1);
  p->compute_slot = make_slot(p.get(), p->compute_points);
  // odf_compute pipeline: the most slots (up to kPipeSlots) of equal size
  // that the workspace holds, each with as many points as fit (at most one
  // batch's worth)
  {
    const int32_t pmax = p->opts.max_batch_points > 0 ? std::min(p->opts.max_batch_points, kMaxBatch) : kMaxBatch;
    int32_t slots = 0, spts = 0;
    for (int ns = kPipeSlots; ns >= 1 && slots == 0; --ns) {
      const int64_t avail = p->opts.workspace_bytes / ns - p->fixed_bytes;
      if (avail < p->per_point_bytes) continue;
      int32_t q = (int32_t)std::min<int64_t>(avail / std::max<int64_t>(p->per_point_bytes, 1), pmax);
      while (q > 1 && (int64_t)ns * make_slot(p.get(), q).bytes > p->opts.workspace_bytes) --q;
      if ((int64_t)ns * make_slot(p.get(), q).bytes <= p->opts.workspace_bytes) {
        slots = ns;
        spts = q;
      }
    }
    if (slots == 0) {   // one point fits (checked above), so this is one slot of one point
      slots = 1;
      spts = 1;
    }
    p->pipe_slots = slots;
    p->pipe_slot = make_slot(p.get(), spts);
    bool ok = hipStreamCreateWithFlags(&p->prep_stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k)
      ok = hipStreamCreateWithFlags(&p->sum_stream[k], hipStreamNonBlocking) == hipSuccess;
    for (int k = 0; k < 3 && ok; ++k)
      ok = hipEventCreateWithFlags(&p->ev_join[k], hipEventDisableTiming) == hipSuccess;
    for (int k = 0; k < slots && ok; ++k)
      ok = hipEventCreateWithFlags(&p->ev_prep[k], hipEventDisableTiming) == hipSuccess &&
           hipEventCreateWithFlags(&p->ev_free[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      set_error("stream or event creation failed");
      release_streams(p.get());
      free_owned(p.get());
      return ODF_E_DEVICE;
    }
  }
  p->loop.reset(new RequestLoop(p.get()));
  *out = p.release();
  return ODF_OK;
}

int64_t odf_point_footprint(const odf_plan_t* plan) { return plan ? plan->per_point_bytes : -1; }

odf_status odf_stage_times(odf_plan_t* plan, double* ms, double* busy_ms, int64_t* launches,
                           int32_t reset) {
  g_err.clear();
  if (!plan || !ms || !busy_ms || !launches) { set_error("odf_stage_times: NULL argument"); return ODF_E_INVALID; }
  std::lock_guard<std::mutex> guard(plan->compute_mu);
  for (int k = 0; k < kStages; ++k) {
    ms[k] = plan->timer.ms[k];
    busy_ms[k] = plan->timer.busy_ms[k];
    launches[k] = plan->timer.launches[k];
    if (reset) {
      plan->timer.ms[k] = 0.0;
      plan->timer.busy_ms[k] = 0.0;
      plan->timer.launches[k] = 0;
    }
  }
  return ODF_OK;
}

odf_status odf_plan_destroy(odf_plan_t* plan) {
  if (!plan) return ODF_OK;
  plan->loop.reset();  // drains and joins the request loop
  (void)hipDeviceSynchronize();
  for (hipEvent_t e : plan->timer.pool) (void)hipEventDestroy(e);
  release_streams(plan);
  if (plan->pinned) (void)hipHostFree(plan->pinned);
  free_owned(plan);
  delete plan;
  return ODF_OK;
}

odf_status odf_compute(odf_plan_t* p, const odf_request* r, odf_stats* stats) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  odf_status st = validate_request(p, r, true);
  if (st != ODF_OK) return st;
  const double t0 = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());   // the request loop is idle while this runs
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  char* base = static_cast<char*>(p->opts.workspace);
  const int NS = p->pipe_slots;
  const SlotLayout& sl = p->pipe_slot;
  const int n = r->n_points;
  const int S = p->n_species;
  // pinned host staging: point arrays and abundances in, counters out
  const size_t need = (size_t)8 * (3 * (size_t)n + S) + 16 * (size_t)std::max(n, 1) + 64;
  if (p->pinned_bytes < need) {
    if (p->pinned) (void)hipHostFree(p->pinned);
    p->pinned = nullptr;
    p->pinned_bytes = 0;
    HIP_TRY(hipHostMalloc(&p->pinned, need, hipHostMallocDefault));
    p->pinned_bytes = need;
  }
  double* hT = static_cast<double*>(p->pinned);
  double* hP = hT + n;
  double* hV = hP + n;
  double* hA = hV + n;
  unsigned long long* h_nsamp = reinterpret_cast<unsigned long long*>(hA + S);
  int32_t* h_nsurv = reinterpret_cast<int32_t*>(h_nsamp + std::max(n, 1));
  int32_t* h_nit = h_nsurv + std::max(n, 1);
  std::memcpy(hT, r->T_K, 8 * (size_t)n);
  std::memcpy(hP, r->log10_P_cgs, 8 * (size_t)n);
  std::memcpy(hV, r->vturb_kms, 8 * (size_t)n);
  std::memcpy(hA, r->abundance, 8 * (size_t)S);
  // fork the pipeline's streams from the caller's stream
  hipStream_t ps = p->prep_stream;
  hipStream_t vs[2] = {p->sum_stream[0], p->sum_stream[1]};
  HIP_TRY(hipEventRecord(p->ev_fork, s));
  HIP_TRY(hipStreamWaitEvent(ps, p->ev_fork, 0));
  HIP_TRY(hipStreamWaitEvent(vs[0], p->ev_fork, 0));
  HIP_TRY(hipStreamWaitEvent(vs[1], p->ev_fork, 0));
  StageTimer* timer = p->opts.kernel_timing ? &p->timer : nullptr;
  auto enqueue_all = [&]() -> odf_status {
    for (int k = 0; k < NS; ++k)
      HIP_TRY(hipMemcpyAsync(base + k * sl.bytes + sl.off_abund, hA, 8 * S, hipMemcpyHostToDevice, ps));
    int batch = 0;
    for (int b0 = 0; b0 < n; b0 += sl.points, ++batch) {
      const int k = batch % NS;
      char* sb = base + k * sl.bytes;
      const int nb = std::min(sl.points, n - b0);
      // preparation, once the slot's previous batch has been reduced
      if (batch >= NS) HIP_TRY(hipStreamWaitEvent(ps, p->ev_free[k], 0));
      HIP_TRY(hipMemcpyAsync(sb + sl.off_T, hT + b0, 8 * nb, hipMemcpyHostToDevice, ps));
      HIP_TRY(hipMemcpyAsync(sb + sl.off_logP, hP + b0, 8 * nb, hipMemcpyHostToDevice, ps));
      HIP_TRY(hipMemcpyAsync(sb + sl.off_vt, hV + b0, 8 * nb, hipMemcpyHostToDevice, ps));
      Batch B = make_batch(p, sl, sb, nb);
      odf_status es = enqueue_prep(p, B, ps, timer);
      if (es != ODF_OK) return es;
      HIP_TRY(hipMemcpyAsync(h_nsurv + b0, B.nsurv, 4 * nb, hipMemcpyDeviceToHost, ps));
      HIP_TRY(hipMemcpyAsync(h_nsamp + b0, B.nsamp, 8 * nb, hipMemcpyDeviceToHost, ps));
      HIP_TRY(hipMemcpyAsync(h_nit + b0, B.nit, 4 * nb, hipMemcpyDeviceToHost, ps));
      HIP_TRY(hipEventRecord(p->ev_prep[k], ps));
      // summation on the summing streams in turn
      hipStream_t v = vs[batch & 1];
      HIP_TRY(hipStreamWaitEvent(v, p->ev_prep[k], 0));
      char* outp = static_cast<char*>(r->out) + (size_t)b0 * out_point_bytes(p);
      es = enqueue_sum(p, B, sb, sl, outp, v, timer);
      if (es != ODF_OK) return es;
      HIP_TRY(hipEventRecord(p->ev_free[k], v));
    }
    return ODF_OK;
  };
  const odf_status est = enqueue_all();
  if (est != ODF_OK) {
    // whatever was enqueued still reads the staging buffers: let it drain
    (void)hipStreamSynchronize(ps);
    (void)hipStreamSynchronize(vs[0]);
    (void)hipStreamSynchronize(vs[1]);
    return est;
  }
  // join back into the caller's stream
  HIP_TRY(hipEventRecord(p->ev_join[0], ps));
  HIP_TRY(hipEventRecord(p->ev_join[1], vs[0]));
  HIP_TRY(hipEventRecord(p->ev_join[2], vs[1]));
  for (hipEvent_t e : p->ev_join) HIP_TRY(hipStreamWaitEvent(s, e, 0));
  HIP_TRY(hipStreamSynchronize(s));
  if (p->opts.kernel_timing) collect_timer(p->timer);
  for (int i = 0; i < n; ++i)
    if (h_nit[i] < 0) {
      set_error("ionisation equilibrium did not converge in %d steps at point %d (T = %g K, log10 P = %g)",
                -h_nit[i], i, r->T_K[i], r->log10_P_cgs[i]);
      return ODF_E_INTERNAL;
    }
  if (stats) {
    std::memset(stats, 0, sizeof *stats);
    stats->state = ODF_DONE;
    stats->t_submit = stats->t_admit = t0;
    stats->t_done = std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
    stats->points = n;
    stats->line_evals = (int64_t)n * p->n_lines;
    for (int i = 0; i < n; ++i) {
      stats->survivors += h_nsurv[i];
      stats->voigt_samples += (int64_t)h_nsamp[i];
    }
  }
  return ODF_OK;
}

// ---- stage entry points ------------------------------------------------------

static odf_status stage_prefix(odf_plan_t* p, const odf_request* r, int32_t point, Batch* B,
                               int rec64, void* rec_override) {
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  char* base = static_cast<char*>(p->opts.workspace);
  const SlotLayout& sl = p->compute_slot;
  HIP_TRY(hipMemcpyAsync(base + sl.off_abund, r->abundance, 8 * p->n_species, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_T, r->T_K + point, 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_logP, r->log10_P_cgs + point, 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_vt, r->vturb_kms + point, 8, hipMemcpyHostToDevice, s));
  *B = make_batch(p, sl, base, 1);
  if (rec_override) B->rec = rec_override;
  HIP_TRY(launch_point_state(s, p->params, *B));
  HIP_TRY(launch_select(s, p->params, p->lines, *B));
  HIP_TRY(launch_scan(s, p->params, p->lines, *B));
  HIP_TRY(launch_emit(s, p->params, p->lines, *B, rec64));
  return ODF_OK;
}

odf_status odf_stage_lines(odf_plan_t* p, const odf_request* r, int32_t point, int64_t* n_surv,
                           int64_t* voigt_samples, int64_t* orig_index, int32_t* j_lo, int32_t* j_hi,
                           double* S, double* a, double* b) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  odf_status st = validate_request(p, r, false);
  if (st != ODF_OK) return st;
  if (point < 0 || point >= r->n_points) { set_error("point %d out of range", point); return ODF_E_INVALID; }
  if (!n_surv || !voigt_samples || !orig_index || !j_lo || !j_hi || !S || !a || !b) {
    set_error("stage_lines: NULL output");
    return ODF_E_INVALID;
  }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  const int64_t L = std::max<int64_t>(p->n_lines, 1);
  Rec64* rec = nullptr;
  if (hipMalloc(&rec, L * sizeof(Rec64)) != hipSuccess) { set_error("hipMalloc failed"); return ODF_E_DEVICE; }
  Batch B;
  st = stage_prefix(p, r, point, &B, 1, rec);
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  int32_t ns = 0;
  unsigned long long nsamp = 0;
  std::vector<Rec64> h;
  if (st == ODF_OK) {
    hipError_t e = hipMemcpyAsync(&ns, B.nsurv, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&nsamp, B.nsamp, 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) {
      h.resize(std::max(ns, 1));
      e = hipMemcpy(h.data(), rec, (size_t)ns * sizeof(Rec64), hipMemcpyDeviceToHost);
    }
    if (e != hipSuccess) {
      set_error("stage_lines copy failed: %s", hipGetErrorString(e));
      st = ODF_E_DEVICE;
    }
  }
  (void)hipFree(rec);
  if (st != ODF_OK) return st;
  // the kernel's order is the narrow class, then the wide one: report the
  // survivors in wavelength order (sorted line index)
  std::sort(h.begin(), h.begin() + ns, [](const Rec64& x, const Rec64& y) { return x.li < y.li; });
  *n_surv = ns;
  *voigt_samples = (int64_t)nsamp;
  for (int i = 0; i < ns; ++i) {
    orig_index[i] = p->orig[h[i].li];
    j_lo[i] = h[i].jlo;
    j_hi[i] = h[i].jhi;
    S[i] = h[i].S;
    a[i] = h[i].y;
    b[i] = p->lnq / h[i].c1;
  }
  return ODF_OK;
}

odf_status odf_stage_records(odf_plan_t* p, const odf_request* r, int32_t point, int64_t* n_surv,
                             int64_t* n_narrow, int32_t* record_bytes, void* rec_host, int64_t capacity,
                             int32_t* wz_host) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  odf_status st = validate_request(p, r, false);
  if (st != ODF_OK) return st;
  if (point < 0 || point >= r->n_points) { set_error("point %d out of range", point); return ODF_E_INVALID; }
  const bool mixed = p->opts.precision == ODF_PREC_MIXED;
  if (!n_surv || !n_narrow || !record_bytes || !rec_host || (mixed && !wz_host)) {
    set_error("stage_records: NULL output");
    return ODF_E_INVALID;
  }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  Batch B;
  if ((st = stage_prefix(p, r, point, &B, mixed ? 0 : 1, nullptr)) != ODF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  int32_t ns = 0, nn = 0;
  HIP_TRY(hipMemcpyAsync(&ns, B.nsurv, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&nn, B.nsurv_n, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t rb = mixed ? (int64_t)sizeof(Rec32) : (int64_t)sizeof(Rec64);
  *n_surv = ns;
  *n_narrow = nn;
  *record_bytes = (int32_t)rb;
  if (ns > capacity) {
    set_error("stage_records: %d survivors, capacity %lld", ns, (long long)capacity);
    return ODF_E_INVALID;
  }
  if (ns > 0) {
    HIP_TRY(hipMemcpy(rec_host, B.rec, (size_t)ns * rb, hipMemcpyDeviceToHost));
    if (mixed) HIP_TRY(hipMemcpy(wz_host, B.wz, (size_t)ns * sizeof(int2), hipMemcpyDeviceToHost));
  }
  return ODF_OK;
}

odf_status odf_debug_set_newton_limit(odf_plan_t* p, int32_t max_steps) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  if (max_steps < 1 || max_steps > 1000) { set_error("max_steps must be in [1, 1000]"); return ODF_E_INVALID; }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  p->params.ne_max_iter = max_steps;
  return ODF_OK;
}

odf_status odf_stage_state(odf_plan_t* p, const odf_request* r, int32_t point, double* state,
                           int32_t* iterations) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  odf_status st = validate_request(p, r, false);
  if (st != ODF_OK) return st;
  if (point < 0 || point >= r->n_points) { set_error("point %d out of range", point); return ODF_E_INVALID; }
  if (!state || !iterations) { set_error("stage_state: NULL output"); return ODF_E_INVALID; }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  char* base = static_cast<char*>(p->opts.workspace);
  const SlotLayout& sl = p->compute_slot;
  HIP_TRY(hipMemcpyAsync(base + sl.off_abund, r->abundance, 8 * p->n_species, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_T, r->T_K + point, 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_logP, r->log10_P_cgs + point, 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(base + sl.off_vt, r->vturb_kms + point, 8, hipMemcpyHostToDevice, s));
  Batch B = make_batch(p, sl, base, 1);
  HIP_TRY(launch_point_state(s, p->params, B));
  PointState ps{};
  int32_t nit = 0;
  HIP_TRY(hipMemcpyAsync(&ps, B.state, sizeof ps, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(&nit, B.nit, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  state[0] = ps.n_e;
  state[1] = ps.n_heavy;
  state[2] = ps.n_H;
  state[3] = ps.rho;
  *iterations = nit;
  return ODF_OK;
}

odf_status odf_stage_fine(odf_plan_t* p, const odf_request* r, int32_t point, void* kappa_dev) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  odf_status st = validate_request(p, r, false);
  if (st != ODF_OK) return st;
  if (point < 0 || point >= r->n_points) { set_error("point %d out of range", point); return ODF_E_INVALID; }
  if (!kappa_dev) { set_error("kappa_dev is NULL"); return ODF_E_INVALID; }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  Batch B;
  const int rec64 = p->opts.precision == ODF_PREC_FP64;
  if ((st = stage_prefix(p, r, point, &B, rec64, nullptr)) != ODF_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  HIP_TRY(launch_voigt(s, p->params, B, p->d_quad));
  const size_t esz = p->opts.precision == ODF_PREC_MIXED ? 4 : 8;
  HIP_TRY(hipMemcpyAsync(kappa_dev, B.kappa, p->N * esz, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return ODF_OK;
}

odf_status odf_stage_reduce(odf_plan_t* p, const void* kappa_dev, void* out_dev) {
  g_err.clear();
  if (!p) { set_error("plan is NULL"); return ODF_E_INVALID; }
  if (!kappa_dev || !out_dev) { set_error("stage_reduce: NULL buffer"); return ODF_E_INVALID; }
  std::lock_guard<std::mutex> guard(p->compute_mu);
  WorkspaceLease lease(p->loop.get());
  hipStream_t s = static_cast<hipStream_t>(p->opts.stream);
  char* base = static_cast<char*>(p->opts.workspace);
  HIP_TRY(launch_odf(s, p->params, kappa_dev, p->N, 1, out_dev, p->odf_classes,
                     base + p->compute_slot.off_gscr, p->d_goff, p->gscr_elems));
  HIP_TRY(hipStreamSynchronize(s));
  return ODF_OK;
}

}  // extern "C"

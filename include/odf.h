/*
 * odf.h - C ABI of the MI355X opacity-distribution-function (ODF) engine.
 *
 * The engine computes, for every (composition, microturbulence, temperature,
 * pressure) point, the line opacity of a line list on a logarithmic
 * wavelength grid of resolving power R and collapses every wavelength bin of
 * that grid into a step function of sub-bin mean opacities: the ODF table of
 * MPS-ATLAS module I (Witzke et al. 2021, "MPS-ATLAS: a fast all-in-one code
 * for synthesising stellar spectra"; Sec. 2.3 "The ODF approach" and App. E
 * "ODF and opacity calculations").
 *
 * Inputs follow the paper's statement of the module-I problem (Sec. 3,
 * module-I inputs of the code-structure figure): elemental composition, a
 * line list, the turbulent velocity, the temperature-pressure grid, the
 * wavelength range and the bin / sub-bin configuration.  Output is the ODF
 * table.  Every computational step runs on the GPU.
 *
 * Conventions
 *   - All functions return odf_status (0 = ODF_OK, < 0 = error).  On error a
 *     message is available from odf_last_error() (thread-local).  No C++
 *     exception crosses this interface.
 *   - "host" pointers are read during the call only and may be freed after it
 *     returns.  "device" pointers are HIP device allocations owned by the
 *     caller (for example PyTorch tensors) and must stay valid for as long as
 *     stated for each field.
 *   - Units are CGS unless stated; wavelengths in nm (vacuum).
 */
#ifndef ODF_H
#define ODF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ODF_OK = 0,
  ODF_E_INVALID = -1,        /* malformed argument; message says which */
  ODF_E_NOMEM = -2,          /* workspace too small for the request */
  ODF_E_DEVICE = -3,         /* a HIP call failed */
  ODF_E_UNKNOWN_TICKET = -4, /* odf_poll/odf_wait on a ticket never issued */
  ODF_E_CANCELLED = -5,      /* plan destroyed while the request waited */
  ODF_E_INTERNAL = -6        /* invariant broken inside the library */
} odf_status;

typedef enum {
  ODF_PREC_FP64 = 0,  /* FP64 everywhere: accurate W(z), FP64 sums, FP64 ODF */
  ODF_PREC_MIXED = 1  /* FP64 line strengths; FP32 Voigt with compensated sums;
                         FP32 sort keys; FP64 step sums; FP32 ODF output */
} odf_precision;

typedef enum {
  ODF_MEAN_GEOMETRIC = 0,  /* sub-bin geometric mean (the paper's default, Sec. 2.3) */
  ODF_MEAN_ARITHMETIC = 1  /* 'odf mean arithmetic' (App. G, module-I keywords) */
} odf_mean;

/* What odf_compute and the request loop write per point. */
typedef enum {
  ODF_OUT_TABLE = 0,  /* the ODF table: [n_bins][n_steps] sub-bin means */
  ODF_OUT_FINE = 1    /* pre-tabulated high-resolution opacity (Sec. 4.1, option to
                         pre-tabulate): the floored line opacity of every fine
                         point, [N] values, i.e. an ODF whose bins are single
                         fine points with one sub-bin; bins and sub-bins of the
                         layout are not used */
} odf_output;

/* How the electron density of a point is found. */
typedef enum {
  ODF_NE_FIXED = 0,       /* P_e = pe_over_p * P */
  ODF_NE_EQUILIBRIUM = 1  /* ionisation equilibrium of hydrogen and every species of
                             the table (App. A, without molecules): Newton-Raphson
                             on the neutral densities and n_e under particle and
                             charge conservation, until every relative change is
                             below 1e-4 */
} odf_electrons;

typedef enum { ODF_PENDING = 0, ODF_RUNNING = 1, ODF_DONE = 2, ODF_FAILED = 3 } odf_state;

/* Line list, structure of arrays, any order (host).  The plan sorts a copy
 * by wavelength and keeps it resident on the device.
 *   lambda_nm    vacuum wavelength of the transition
 *   log_gf       log10 of g_i f_ij (Sec. 2.1, eq. l_nu_line)
 *   e_low_ev     energy of the lower level E_i
 *   species      0..n_species-1;  stage 0..n_stages-1 (0 = neutral)
 *   log_g_rad    log10 radiative damping [s^-1]
 *   log_g_stark  log10 quadratic-Stark damping per electron at 10^4 K [s^-1 cm^3]
 *   log_g_vdw    log10 van der Waals damping per heavy particle at 10^4 K [s^-1 cm^3]
 * The total damping constant (Sec. 2.1) is
 *   gamma = g_rad + g_stark n_e (T/1e4)^(1/6) + g_vdw N_heavy (T/1e4)^0.3. */
typedef struct {
  int64_t n_lines;
  const double *lambda_nm, *log_gf, *e_low_ev;
  const int32_t *species, *stage;
  const double *log_g_rad, *log_g_stark, *log_g_vdw;
} odf_lines;

/* Species table (host).
 *   mass_amu  [n_species]                  atomic mass (Doppler width, App. E)
 *   chi_ev    [n_species][n_stages-1]      ionisation energy of stage k -> k+1
 *   part_fn   [n_species][n_stages]        partition function U_k (T-independent) */
typedef struct {
  int32_t n_species, n_stages;
  const double *mass_amu, *chi_ev, *part_fn;
} odf_species;

/* Wavelength grid and bin / sub-bin layout (host).
 * Fine grid: lambda_j = lambda_first_nm * (1 + 1/R)^j, j = 0..N-1, N the
 * number of points not beyond lambda_last_nm (App. E grid formula, 0-based).
 *   bin_edges [n_bins+1] fine indices, strictly increasing, 0 <= e < = N.
 *             Bin b covers [bin_edges[b], bin_edges[b+1]); any width
 *             1..20000 points is accepted (user-defined binning, App. E).
 *   step_frac [n_steps] sub-bin widths as fractions of the bin, > 0, summing
 *             to 1 within 1e-9, listed from the lowest opacity upward. */
typedef struct {
  double lambda_first_nm, lambda_last_nm, resolving_power;
  int32_t n_bins;
  const int64_t *bin_edges;
  int32_t n_steps;
  const double *step_frac;
} odf_layout;

/* Plan options.
 *   cutoff            line pre-selection factor (Sec. 4.3): a line is kept if
 *                     its core opacity S*H(0,a) >= cutoff*kappa_c(lambda_0);
 *                     its window ends where its envelope drops below that
 *                     level; the fine-grid opacity is floored at it.
 *   window_cap_doppler cap of the half-window in Doppler widths.
 *   pe_over_p         electron pressure as a fraction of the gas pressure
 *                     (electrons = ODF_NE_FIXED; ignored otherwise).
 *   kappa_c_*         continuum kappa_c(lambda) = ref * (lambda/lambda_ref)^power [cm^2/g].
 *   workspace         caller-owned device memory used for all intermediate
 *                     data; must outlive the plan.  Its size bounds the number
 *                     of points processed together and the number of requests
 *                     the request loop admits at once.
 *   stream            hipStream_t used by odf_compute (NULL = default stream).
 *   max_batch_points  upper bound on points per device batch (0 = automatic).
 *   loop_streams      streams used by the request loop (0 = 2).
 *   kernel_timing     nonzero: odf_compute brackets every kernel launch with
 *                     HIP events on options.stream; totals are read with
 *                     odf_stage_times().
 *   output            odf_output: ODF table (default) or fine-grid opacity.
 *   electrons         odf_electrons: fixed P_e / P (default) or the
 *                     ionisation equilibrium.  With the equilibrium, a point
 *                     whose Newton iteration does not converge within 100
 *                     steps fails its request (odf_compute returns
 *                     ODF_E_INTERNAL naming the point; a ticket ends FAILED). */
typedef struct {
  odf_precision precision;
  odf_mean mean;
  double cutoff;
  double window_cap_doppler;
  double pe_over_p;
  double kappa_c_ref, lambda_c_ref_nm, kappa_c_power;
  void *workspace;
  int64_t workspace_bytes;
  void *stream;
  int32_t max_batch_points;
  int32_t loop_streams;
  int32_t kernel_timing;
  int32_t output;
  int32_t electrons;
} odf_options;

/* One ODF request.
 *   abundance  host [n_species] number ratio N_s/N_H, > 0
 *   T_K, log10_P_cgs, vturb_kms  host [n_points] point list (a T-P grid and a
 *              list of microturbulences, App. G 'velocities values' and the
 *              odf.tpgrid file, expanded by the caller)
 *   out        device buffer [n_points][n_bins][n_steps] (ODF_OUT_TABLE) or
 *              [n_points][N] (ODF_OUT_FINE) of double (FP64) or float
 *              (MIXED), caller-owned, written in full; valid once
 *              odf_compute returns or odf_poll reports ODF_DONE. */
typedef struct {
  const double *abundance;
  int32_t n_points;
  const double *T_K, *log10_P_cgs, *vturb_kms;
  void *out;
} odf_request;

/* Per-request statistics.  Times are seconds on a monotonic clock.
 *   line_evals    lines considered, summed over points (selection included)
 *   survivors     kept lines with a non-empty window, summed over points
 *   voigt_samples profile samples added to the grid, summed over points */
typedef struct {
  odf_state state;
  double t_submit, t_admit, t_done;
  int64_t points, line_evals, survivors, voigt_samples;
  char msg[128];
} odf_stats;

/* State of a plan's request loop (odf_loop_status).  The workspace is the
 * loop's byte pool; a request reserves its footprint (odf_request_footprint)
 * from it when admitted and releases it when final.
 *   pool_bytes              the pool (the workspace, rounded down to 256 B)
 *   resident_bytes          bytes reserved by the admitted requests now
 *   peak_resident_bytes     the most ever reserved at once
 *   resident_requests       admitted and not yet final
 *   peak_resident_requests  the most ever resident at once
 *   queued_requests         submitted, waiting for room
 *   batches_in_flight       batches on the device now
 *   slot_points             points per batch slot of a request of that many points or more
 *   slots_per_request       batch slots a request reserves (at most) */
typedef struct {
  int64_t pool_bytes, resident_bytes, peak_resident_bytes;
  int32_t resident_requests, peak_resident_requests, queued_requests, batches_in_flight;
  int32_t slot_points, slots_per_request;
} odf_loop_info;

typedef struct odf_plan_s odf_plan_t;

/* Build a plan: validates and copies every host array, sorts the lines by
 * wavelength, uploads them and the per-line constants (App. E first stage,
 * items i-iii, per line) and sizes the workspace.  *out receives the plan.
 * Errors: ODF_E_INVALID (bad argument), ODF_E_NOMEM (workspace smaller than
 * one point needs), ODF_E_DEVICE. */
odf_status odf_plan(const odf_lines *lines, const odf_species *species,
                    const odf_layout *layout, const odf_options *opts,
                    odf_plan_t **out);

/* Compute one request on options.stream and wait for it (App. E, stages one
 * to three for every point).  The points go in batches through up to four
 * slots of the workspace: an internal preparation stream runs the line
 * selection of upcoming batches while two internal summing streams run the
 * Voigt sums and ODF reductions of earlier ones; all three are ordered after
 * the work already on options.stream, and options.stream waits for them
 * before this returns.  Results do not depend on the batching.  Must not run
 * concurrently with another odf_compute on the same plan; the request loop
 * pauses while it runs.  stats may be NULL. */
odf_status odf_compute(odf_plan_t *plan, const odf_request *req, odf_stats *stats);

/* Queue a request for the plan's request loop and return at once.  The host
 * arrays are copied; req->out must stay valid until the ticket is final.
 * The request's device work is ordered after the work queued on
 * options.stream when it is submitted (req->out may have been allocated
 * there).  Admission is by HBM footprint: the workspace is a byte pool, and
 * the oldest waiting request is admitted as soon as its footprint
 * (odf_request_footprint: up to two batch slots of min(n_points, 16)
 * points) fits the free bytes; it keeps them until it is final, and later
 * requests never overtake it.  Resident requests take turns handing one
 * batch each to the device.  ODF_E_NOMEM if the footprint exceeds the whole
 * pool, so that the request could never be admitted. */
odf_status odf_submit(odf_plan_t *plan, const odf_request *req, int64_t *ticket);

/* Non-blocking status of a ticket; DONE and FAILED are final. */
odf_status odf_poll(odf_plan_t *plan, int64_t ticket, odf_stats *out);

/* Block until the ticket is final or timeout_s elapses (then ODF_OK with
 * out->state still PENDING or RUNNING). */
odf_status odf_wait(odf_plan_t *plan, int64_t ticket, double timeout_s, odf_stats *out);

/* Drain the request loop, free device memory owned by the plan.  NULL-safe;
 * a second call on the same pointer is not allowed (the plan is freed). */
odf_status odf_plan_destroy(odf_plan_t *plan);

/* Number of fine-grid points N of a layout (App. E grid formula), or -1. */
int64_t odf_grid_points(const odf_layout *layout);

/* Workspace bytes that one point occupies while it is being processed. */
int64_t odf_point_footprint(const odf_plan_t *plan);

/* Workspace bytes the request loop reserves for a request of n_points
 * while it is resident (0 for no points, -1 for a NULL plan). */
int64_t odf_request_footprint(const odf_plan_t *plan, int32_t n_points);

/* Current and peak occupancy of the request loop's pool (odf_loop_info).
 * ODF_E_INVALID for a NULL argument. */
odf_status odf_loop_status(odf_plan_t *plan, odf_loop_info *out);

/* Message of the last error on this thread ("" if none). */
const char *odf_last_error(void);

/* ---- stage entry points, for checking each kernel on its own ---------- */

/* Line-strength stage for point `point` of req: pre-selection, strength,
 * damping and window of every line (Sec. 2.1 eq. l_nu_line; Sec. 4.3; App. E).
 * Host outputs, each of capacity plan line count, in wavelength order of
 * survivors: orig_index (index into the caller's line list), j_lo, j_hi,
 * S [cm^2/g], a, b (= dnu_D/nu_0).  *n_surv receives the survivor count;
 * *voigt_samples the sum of window lengths. */
odf_status odf_stage_lines(odf_plan_t *plan, const odf_request *req, int32_t point,
                           int64_t *n_surv, int64_t *voigt_samples,
                           int64_t *orig_index, int32_t *j_lo, int32_t *j_hi,
                           double *S, double *a, double *b);

/* Survivor records of point `point` of req exactly as this plan's Voigt
 * kernel reads them, for checking the values the kernel trusts.  Order: the
 * *n_narrow survivors whose half-window (the larger side from the nearest
 * grid index of the centre, plus one) is at most 1024 fine points, then the
 * others, each class in wavelength order.  MIXED plans: 48-byte FP32
 * records (int32 J = nearest index of the line centre, j_lo, j_hi, packed
 * zone half-widths; float phi = centre - J, c1 = sigma ln q / b, the
 * far-wing fraction S H = (A v + B) / (v^2 + E) with v = u^2 + D and
 * u = sigma x, S, a; sigma = 1, or 1/a in the Lorentz limit a >= 1e4),
 * and in wz_host [2 n_surv] the (J, packed zone half-widths) pairs read
 * beside the windows; the zone half-widths are the fine points around J
 * where |x| < 15 (low 16 bits) and |x| < 6 (high 16 bits) may occur,
 * -32768 for none.  FP64 plans: 64-byte records (J, j_lo, j_hi, zone
 * half-widths for |x| < 8 and < 40 or -1, sorted line index, two pads;
 * double phi, S, a, c1 = ln q / b); wz_host is not used and may be NULL.
 *   rec_host  host buffer of `capacity` records; *n_surv receives the
 *             survivor count and *record_bytes the record size.
 * ODF_E_INVALID when more than `capacity` lines survive (the count is
 * still returned). */
odf_status odf_stage_records(odf_plan_t *plan, const odf_request *req, int32_t point,
                             int64_t *n_surv, int64_t *n_narrow, int32_t *record_bytes,
                             void *rec_host, int64_t capacity, int32_t *wz_host);

/* Gas state of point `point` of req (Sec. 2.1; App. A): state host [4]
 * receives n_e, the heavy-particle density N_heavy = P/kT - n_e (with fixed
 * P_e: (P - P_e)/kT), the hydrogen density N_H [cm^-3] and the mass density
 * rho [g cm^-3]; *iterations the Newton steps of the ionisation equilibrium
 * (0 with fixed P_e, negative if it did not converge). */
odf_status odf_stage_state(odf_plan_t *plan, const odf_request *req, int32_t point,
                           double *state, int32_t *iterations);

/* Line opacity on the fine grid for point `point` (before the floor):
 * kappa_dev is a device buffer of N doubles (FP64 plan) or floats (MIXED). */
odf_status odf_stage_fine(odf_plan_t *plan, const odf_request *req, int32_t point,
                          void *kappa_dev);

/* ODF reduction of one fine grid (floor, per-bin sort, sub-bin means):
 * kappa_dev device [N] (double for FP64 plans, float for MIXED), out_dev
 * device [n_bins][n_steps] (same type).  Runs on options.stream and waits. */
odf_status odf_stage_reduce(odf_plan_t *plan, const void *kappa_dev, void *out_dev);

/* Kernel times accumulated by odf_compute when options.kernel_timing is set,
 * per stage: 0 point state, 1 line selection, 2 survivor scan, 3 survivor
 * emission, 4 Voigt scatter-sum, 5 ODF reduction.  All arrays are host
 * [6], caller-owned.  ms receives the summed HIP-event durations of the
 * launches in milliseconds; busy_ms the length of the union of their
 * intervals (less than ms when odf_compute's internal streams run
 * launches of one stage at the same time); launches the launch counts.
 * reset nonzero clears the totals afterwards.  ODF_E_INVALID for a NULL
 * argument. */
odf_status odf_stage_times(odf_plan_t *plan, double *ms, double *busy_ms, int64_t *launches,
                           int32_t reset);

/* ---- allocation-free entry point -------------------------------------- */

/* For callers that cannot allocate device memory or wait (code under HIP
 * graph capture, serving loops that forbid allocation): the ODF reduction
 * of odf_stage_reduce (floor, per-bin sort, sub-bin means) over n_points
 * fine grids, enqueued on `stream` (NULL: options.stream) and not waited
 * for.  It calls no allocator: bins too large for LDS sort in a static
 * device array of the library, 32 MiB per GPU (held until the process
 * ends), instead of the plan's workspace.
 *   kappa_dev  device [n_points][N], float (MIXED plan) or double (FP64),
 *              read only; caller-owned, valid until the work completes
 *   out_dev    device [n_points][n_bins][n_steps] of the same type, written
 *              in full once the stream reaches this work
 * Must be called with the plan's device current.  Every call on one GPU,
 * from any plan, shares that GPU's array and keeps what the last call left
 * there: two calls whose work overlaps on the device (on different streams)
 * race, and the caller must order them.  odf_compute, the request loop and
 * odf_stage_reduce do not use the array.  Nothing in it needs clearing:
 * each call writes every scratch key before it reads it.
 * Errors: ODF_E_INVALID (NULL plan or buffer, n_points outside [0, 65535],
 * a plan with output = fine, another device current), ODF_E_NOMEM when the
 * oversize bins of n_points grids need more scratch than the array holds
 * (odf_noalloc_scratch_need), ODF_E_DEVICE on a launch error. */
odf_status odf_reduce_noalloc(odf_plan_t *plan, const void *kappa_dev, int32_t n_points,
                              void *out_dev, void *stream);

/* Bytes of static scratch that odf_reduce_noalloc needs for n_points grids
 * of this plan (0 when every bin fits LDS), or -1 for a NULL plan or
 * negative count. */
int64_t odf_noalloc_scratch_need(const odf_plan_t *plan, int32_t n_points);

/* Test hook for failure handling: the next batch of `ticket` that the
 * request loop launches reports a launch error instead of running, so the
 * ticket ends FAILED while every other ticket completes normally. */
odf_status odf_debug_fail_next_batch(odf_plan_t *plan, int64_t ticket);

/* Test hook for failure handling: the ionisation equilibrium of this plan
 * may take at most max_steps Newton steps (1..1000; 100 by default), so a
 * test can make points fail to converge from the host.  Waits for the
 * request loop to be idle.  ODF_E_INVALID for a NULL plan or a bad count. */
odf_status odf_debug_set_newton_limit(odf_plan_t *plan, int32_t max_steps);

#ifdef __cplusplus
}
#endif

#endif /* ODF_H */

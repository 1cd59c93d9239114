// Host-side plan object of the ODF engine (private).
#pragma once

#include <atomic>
#include <condition_variable>
#include <cstdarg>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/odf.h"
#include "odf_internal.h"

namespace odf {

QuadConsts make_quad_consts();
void set_error(const char* fmt, ...);
std::string g_last_error_copy();
void g_last_error_clear();

// Layout of one batch slot inside the workspace.
struct SlotLayout {
  int64_t off_T, off_logP, off_vt, off_abund, off_state, off_pop, off_bT, off_keep, off_wline, off_blk,
      off_nsurv, off_nsurv_n, off_hmax, off_hmax_w, off_nsamp, off_nit, off_rec, off_win, off_wz,
      off_kappa, off_gscr;
  int64_t bytes;      // total bytes of the slot
  int32_t points;     // points per slot
};

// Slots of the odf_compute pipeline (at most).
constexpr int kPipeSlots = 4;

// Newton steps allowed to the ionisation equilibrium of a point.
constexpr int kNeMaxSteps = 100;

// Size of the static device array that odf_reduce_noalloc sorts oversize
// bins in (one copy per GPU, held until the process ends).
constexpr int64_t kNoAllocScratchBytes = 32ll << 20;
// Device address of that array on device `dev`, resolved once per device
// (noalloc.hip); nullptr with the error set on failure.
void* noalloc_scratch(int dev);

// HIP-event timing of the kernels that odf_compute launches (opt-in).
constexpr int kStages = 6;
struct StageTimer {
  std::vector<hipEvent_t> pool;      // event pairs, reused between calls
  std::vector<int> stage_of_pair;    // stage of each recorded pair
  size_t used = 0;                   // pairs recorded since the last collect
  double ms[kStages] = {0, 0, 0, 0, 0, 0};       // summed launch durations
  double busy_ms[kStages] = {0, 0, 0, 0, 0, 0};  // union of the launch intervals
  int64_t launches[kStages] = {0, 0, 0, 0, 0, 0};
};

struct Request;       // request-loop entry (loop.cpp)
class RequestLoop;    // (loop.cpp)

}  // namespace odf

struct odf_plan_s {
  // validated copies
  odf_options opts{};
  int device = -1;                  // HIP device current when the plan was built
  int32_t n_species = 0, n_stages = 0;
  int64_t n_lines = 0, N = 0;
  int32_t n_bins = 0, n_steps = 0;
  int32_t max_bin = 0;
  double lambda_first_nm = 0, lambda_last_nm = 0, resolving_power = 0, lnq = 0;
  std::vector<int64_t> edges;
  std::vector<double> Fcum;
  std::vector<int64_t> orig;        // sorted position -> caller's line index

  // device allocations owned by the plan
  std::vector<void*> owned;
  odf::DevLines lines{};
  odf::Params params{};
  odf::QuadConsts quad{};
  odf::QuadConsts* d_quad = nullptr;   // device copy read by the Voigt kernels
  int64_t* d_goff = nullptr;        // per-bin offsets into the ODF global scratch
  odf::OdfClasses odf_classes{};    // bins grouped by padded size
  int64_t gscr_elems = 0;           // scratch elements per point

  // workspace carving
  int64_t per_point_bytes = 0;
  int64_t fixed_bytes = 0;
  int32_t compute_points = 0;       // points per odf_compute batch
  odf::SlotLayout compute_slot{};   // one batch of compute_points (stage entry points)
  // odf_compute pipeline: `pipe_slots` slots of `pipe_slot.points` points.
  // A preparation stream fills slot b % pipe_slots with batch b (point
  // state, selection, scan, emission) as soon as the slot is free; two
  // summing streams take the batches alternately (Voigt scatter-sum, ODF
  // reduction).  All three fork from and join back to options.stream, so the
  // Voigt kernels of consecutive batches overlap each other's tails and the
  // next batches' preparation never waits behind a Voigt kernel.
  int32_t pipe_slots = 1;
  odf::SlotLayout pipe_slot{};
  hipStream_t prep_stream = nullptr;
  hipStream_t sum_stream[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
  hipEvent_t ev_prep[odf::kPipeSlots] = {};   // batch of the slot prepared
  hipEvent_t ev_free[odf::kPipeSlots] = {};   // slot summed and reduced
  void* pinned = nullptr;           // host staging of point arrays and counters
  size_t pinned_bytes = 0;

  odf::StageTimer timer;
  std::mutex compute_mu;
  std::unique_ptr<odf::RequestLoop> loop;
};

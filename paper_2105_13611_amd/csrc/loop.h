// Continuous-batching request loop of the ODF engine (private).
//
// One host thread owns every launch.  Submitted requests wait in a FIFO
// queue; a request is admitted as soon as a batch slot of the workspace is
// free and fewer than the maximum number of requests are resident.  Slots
// are handed out round-robin over the resident requests, one batch of
// points at a time, on several HIP streams, so batches of different
// requests (different compositions and point sets) are on the device
// together.  Completion is detected with HIP events; every batch is
// computed independently of what else runs, so a request's result does not
// depend on the mix it ran in.
#pragma once

#include "plan.h"
#include "scheduler.h"

namespace odf {

SlotLayout make_slot(const odf_plan_s* p, int32_t pts);
Batch make_batch(const odf_plan_s* p, const SlotLayout& s, char* base, int32_t n_points);
// The per-batch chain: preparation (point state, selection, scan, survivor
// emission) then summation (Voigt scatter-sum, ODF reduction into `out`).
odf_status enqueue_prep(odf_plan_s* p, const Batch& B, hipStream_t st, StageTimer* timer = nullptr);
odf_status enqueue_sum(odf_plan_s* p, const Batch& B, char* slot_base, const SlotLayout& s,
                       void* out, hipStream_t st, StageTimer* timer = nullptr);
odf_status enqueue_batch(odf_plan_s* p, const Batch& B, char* slot_base, const SlotLayout& s,
                         void* out, hipStream_t st, StageTimer* timer = nullptr);
odf_status validate_request(const odf_plan_s* p, const odf_request* r, bool need_out);
// Bytes of one point's output (ODF table or fine-grid opacity).
size_t out_point_bytes(const odf_plan_s* p);

struct Request {
  int64_t id = 0;
  std::vector<double> abundance, T, logP, vt;
  void* out = nullptr;
  int32_t n_points = 0;
  int32_t next = 0;        // first point not yet dispatched
  int32_t done = 0;        // points completed
  int32_t inflight = 0;    // batches on the device
  bool failed = false;
  bool force_fail = false; // test hook: the next batch launch reports an error
  odf_stats stats{};
};

struct Slot {
  char* base = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  double* h_pts = nullptr;             // pinned staging: T, logP, vt, abundance
  int32_t* h_nsurv = nullptr;          // pinned read-back
  unsigned long long* h_nsamp = nullptr;
  int32_t* h_nit = nullptr;            // ionisation-equilibrium steps per point
  std::shared_ptr<Request> req;
  int32_t first = 0, count = 0;
  bool busy = false;
};

class RequestLoop {
 public:
  explicit RequestLoop(odf_plan_s* p);
  ~RequestLoop();
  odf_status submit(const odf_request* r, int64_t* ticket);
  odf_status poll(int64_t ticket, odf_stats* out);
  odf_status wait(int64_t ticket, double timeout_s, odf_stats* out);
  odf_status fail_next_batch(int64_t ticket);
  int64_t footprint(int32_t n_points) const;
  void acquire_exclusive();
  void release_exclusive();
  int32_t slot_points() const { return layout_.points; }
  int32_t n_slots() const { return (int32_t)slots_.size(); }

 private:
  void run();
  bool start_locked();          // lazily creates streams, events and pinned buffers
  void dispatch_locked(Slot& s, const std::shared_ptr<Request>& r);
  void finish_locked(Slot& s, bool ok, const char* msg);
  static double now();

  odf_plan_s* plan_;
  SlotLayout layout_{};
  std::vector<Slot> slots_;
  std::vector<hipStream_t> streams_;
  std::mutex mu_;
  std::condition_variable cv_;
  BatchScheduler<Request> sched_{16};                // admission and batch hand-out
  std::map<int64_t, std::shared_ptr<Request>> all_;   // every ticket
  int64_t next_id_ = 1;
  bool stop_ = false;
  bool started_ = false;
  bool start_failed_ = false;
  int exclusive_ = 0;
  std::thread th_;
};

struct WorkspaceLease {
  RequestLoop* l;
  explicit WorkspaceLease(RequestLoop* loop) : l(loop) { if (l) l->acquire_exclusive(); }
  ~WorkspaceLease() { if (l) l->release_exclusive(); }
};

}  // namespace odf

// Continuous-batching request loop of the ODF engine (private).
//
// One host thread owns every launch.  Submitted requests wait in a FIFO
// queue.  The workspace is a byte pool: a request is admitted when its
// footprint - batch slots of its own, up to two of min(n, 16) points - fits
// the free bytes, in arrival order, and releases it when it completes or
// fails.  The resident requests take turns (round-robin) handing one batch
// of points at a time into a free slot of their own; slots run on several
// HIP streams, so batches of different requests (different compositions
// and point sets) are on the device together.  A batch holds nothing in its
// slot once it is done: points are staged and counters read back per batch.
// Completion is signalled by a host function queued behind each batch's
// event (a timed wait covers a lost signal); every batch is computed
// independently of what else runs, so a request's result does not depend on
// the mix it ran in.
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

// Points per slot of the request loop (requests with fewer points get
// slots of their size), slots per request, and batches that may be in flight
// at once (each has pinned staging and an event).
constexpr int32_t kLoopSlotPoints = 16;
constexpr int32_t kSlotsPerRequest = 2;
constexpr int kBatchContexts = 64;

// A batch slot of a resident request.
struct Slot {
  char* base = nullptr;
  hipStream_t stream = nullptr;
  int ctx = -1;                 // batch context while busy
  int32_t first = 0, count = 0; // points of the batch in flight
  bool busy = false;
  bool failed = false;          // its dispatch failed after part of it was enqueued
  char msg[128] = {0};
};

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
  hipEvent_t ready = nullptr;   // recorded on options.stream at submit
  // footprint reserved from the pool at admission
  int64_t region = -1, region_bytes = 0;
  SlotLayout layout{};          // one of its slots
  std::vector<Slot> slots;
  int free_slot() const {
    for (size_t i = 0; i < slots.size(); ++i)
      if (!slots[i].busy) return (int)i;
    return -1;
  }
};

// Pinned staging and completion event of one batch in flight.
struct BatchCtx {
  hipEvent_t done = nullptr;
  double* h_pts = nullptr;      // T, log P, v_turb (slot_points each), abundance
  int32_t* h_nsurv = nullptr;
  unsigned long long* h_nsamp = nullptr;
  int32_t* h_nit = nullptr;
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
  void info(odf_loop_info* out);
  void acquire_exclusive();
  void release_exclusive();

 private:
  void run();
  bool start_locked();          // lazily creates streams, batch contexts and the thread
  bool reserve_locked(const std::shared_ptr<Request>& r);
  void dispatch_locked(std::unique_lock<std::mutex>& lk, const std::shared_ptr<Request>& r, int slot);
  void finish_locked(const std::shared_ptr<Request>& r, Slot& s, bool ok, const char* msg);
  static void wake(void* self);
  static double now();

  odf_plan_s* plan_;
  int32_t slot_points_ = 1;     // points per slot of a request with that many or more
  int32_t max_slots_ = 1;       // slots per request
  BytePool pool_;
  std::vector<BatchCtx> ctx_;
  std::vector<int> free_ctx_;
  void* arena_ = nullptr;       // pinned memory of the batch contexts
  std::vector<hipStream_t> streams_;
  size_t next_stream_ = 0;
  std::mutex mu_;
  std::condition_variable cv_;
  BatchScheduler<Request> sched_;                     // admission and batch hand-out
  std::map<int64_t, std::shared_ptr<Request>> all_;   // every ticket
  int64_t next_id_ = 1;
  int32_t inflight_ = 0;
  int32_t peak_resident_ = 0;
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

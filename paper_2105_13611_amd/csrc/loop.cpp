// Continuous-batching request loop (see loop.h).
#include "loop.h"

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>

namespace odf {

double RequestLoop::now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

RequestLoop::RequestLoop(odf_plan_s* p) : plan_(p) {
  const int64_t ws = p->opts.workspace_bytes;
  int32_t pts = std::max<int32_t>(1, std::min<int32_t>(p->compute_points, kLoopSlotPoints));
  while (pts > 1 && make_slot(p, pts).bytes * kSlotsPerRequest > ws) pts = std::max(1, pts / 2);
  slot_points_ = pts;
  const int64_t fit = ws / std::max<int64_t>(make_slot(p, pts).bytes, 1);
  max_slots_ = (int32_t)std::max<int64_t>(1, std::min<int64_t>(fit, kSlotsPerRequest));
  pool_.reset(ws, 256);
}

RequestLoop::~RequestLoop() {
  {
    std::unique_lock<std::mutex> lk(mu_);
    stop_ = true;
    for (auto& r : sched_.waiting()) {
      r->stats.state = ODF_FAILED;
      r->stats.t_done = now();
      std::snprintf(r->stats.msg, sizeof r->stats.msg, "cancelled: plan destroyed before admission");
    }
    sched_.waiting().clear();
    cv_.notify_all();
  }
  if (th_.joinable()) th_.join();
  // host functions queued behind the last batches may still be running
  for (auto st : streams_) (void)hipStreamSynchronize(st);
  for (auto& kv : all_)
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
  for (auto& c : ctx_)
    if (c.done) (void)hipEventDestroy(c.done);
  if (arena_) (void)hipHostFree(arena_);
  for (auto st : streams_) (void)hipStreamDestroy(st);
}

bool RequestLoop::start_locked() {
  if (started_) return !start_failed_;
  started_ = true;
  const int ns = std::max(1, (int)plan_->opts.loop_streams);
  for (int i = 0; i < ns; ++i) {
    hipStream_t s = nullptr;
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      set_error("request loop: hipStreamCreate failed");
      start_failed_ = true;
      return false;
    }
    streams_.push_back(s);
  }
  // pinned staging of every batch context, one arena
  const int32_t P = slot_points_, S = plan_->n_species;
  auto al = [](size_t b) { return (b + 63) / 64 * 64; };
  const size_t b_pts = al(sizeof(double) * (3 * (size_t)P + S)), b_surv = al(4 * (size_t)P),
               b_samp = al(8 * (size_t)P), b_nit = al(4 * (size_t)P);
  const size_t per = b_pts + b_surv + b_samp + b_nit;
  if (hipHostMalloc(&arena_, per * kBatchContexts, hipHostMallocDefault) != hipSuccess) {
    arena_ = nullptr;
    set_error("request loop: pinned staging allocation failed");
    start_failed_ = true;
    return false;
  }
  ctx_.resize(kBatchContexts);
  for (int i = 0; i < kBatchContexts; ++i) {
    char* b = static_cast<char*>(arena_) + per * i;
    BatchCtx& c = ctx_[i];
    c.h_pts = reinterpret_cast<double*>(b);
    c.h_nsurv = reinterpret_cast<int32_t*>(b + b_pts);
    c.h_nsamp = reinterpret_cast<unsigned long long*>(b + b_pts + b_surv);
    c.h_nit = reinterpret_cast<int32_t*>(b + b_pts + b_surv + b_samp);
    if (hipEventCreateWithFlags(&c.done, hipEventDisableTiming) != hipSuccess) {
      set_error("request loop: event creation failed");
      start_failed_ = true;
      return false;
    }
    free_ctx_.push_back(kBatchContexts - 1 - i);
  }
  th_ = std::thread([this] { run(); });
  return true;
}

int64_t RequestLoop::footprint(int32_t n_points) const {
  const RequestShape sh = request_shape(n_points, slot_points_, max_slots_);
  if (sh.slots == 0) return 0;
  return make_slot(plan_, sh.slot_points).bytes * sh.slots;
}

odf_status RequestLoop::submit(const odf_request* r, int64_t* ticket) {
  odf_status st = validate_request(plan_, r, true);
  if (st != ODF_OK) return st;
  if (!ticket) { set_error("ticket is NULL"); return ODF_E_INVALID; }
  const int64_t need = footprint(r->n_points);
  if (need > pool_.capacity()) {
    set_error("request of %d points needs %lld workspace bytes, the pool holds %lld", r->n_points,
              (long long)need, (long long)pool_.capacity());
    return ODF_E_NOMEM;
  }
  auto q = std::make_shared<Request>();
  const int S = plan_->n_species, n = r->n_points;
  q->abundance.assign(r->abundance, r->abundance + S);
  q->T.assign(r->T_K, r->T_K + n);
  q->logP.assign(r->log10_P_cgs, r->log10_P_cgs + n);
  q->vt.assign(r->vturb_kms, r->vturb_kms + n);
  q->out = r->out;
  q->n_points = n;
  q->stats.state = ODF_PENDING;
  q->stats.points = n;
  // the request's work is ordered after what the caller has queued on
  // options.stream so far (its output buffer may have been allocated there)
  hipError_t e = hipEventCreateWithFlags(&q->ready, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(q->ready, static_cast<hipStream_t>(plan_->opts.stream));
  if (e != hipSuccess) {
    if (q->ready) (void)hipEventDestroy(q->ready);
    set_error("submit: event on options.stream failed: %s", hipGetErrorString(e));
    return ODF_E_DEVICE;
  }
  std::unique_lock<std::mutex> lk(mu_);
  if (stop_ || !start_locked()) {
    (void)hipEventDestroy(q->ready);
    if (stop_) { set_error("plan is being destroyed"); return ODF_E_CANCELLED; }
    return ODF_E_DEVICE;
  }
  q->id = next_id_++;
  q->stats.t_submit = now();
  all_[q->id] = q;
  sched_.enqueue(q);
  *ticket = q->id;
  cv_.notify_all();
  return ODF_OK;
}

odf_status RequestLoop::poll(int64_t ticket, odf_stats* out) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) { set_error("unknown ticket %lld", (long long)ticket); return ODF_E_UNKNOWN_TICKET; }
  if (out) *out = it->second->stats;
  return ODF_OK;
}

odf_status RequestLoop::wait(int64_t ticket, double timeout_s, odf_stats* out) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) { set_error("unknown ticket %lld", (long long)ticket); return ODF_E_UNKNOWN_TICKET; }
  auto r = it->second;
  const auto deadline = std::chrono::steady_clock::now() +
                        std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                            std::chrono::duration<double>(std::max(0.0, timeout_s)));
  cv_.wait_until(lk, deadline, [&] {
    return r->stats.state == ODF_DONE || r->stats.state == ODF_FAILED;
  });
  if (out) *out = r->stats;
  return ODF_OK;
}

odf_status RequestLoop::fail_next_batch(int64_t ticket) {
  std::unique_lock<std::mutex> lk(mu_);
  auto it = all_.find(ticket);
  if (it == all_.end()) { set_error("unknown ticket %lld", (long long)ticket); return ODF_E_UNKNOWN_TICKET; }
  it->second->force_fail = true;
  return ODF_OK;
}

void RequestLoop::info(odf_loop_info* out) {
  std::unique_lock<std::mutex> lk(mu_);
  out->pool_bytes = pool_.capacity();
  out->resident_bytes = pool_.used();
  out->peak_resident_bytes = pool_.peak();
  out->resident_requests = (int32_t)sched_.resident();
  out->peak_resident_requests = peak_resident_;
  out->queued_requests = (int32_t)sched_.waiting().size();
  out->batches_in_flight = inflight_;
  out->slot_points = slot_points_;
  out->slots_per_request = max_slots_;
}

void RequestLoop::acquire_exclusive() {
  std::unique_lock<std::mutex> lk(mu_);
  ++exclusive_;
  cv_.notify_all();
  // the resident requests' slots hold nothing between batches, so the
  // workspace is free once no batch is in flight
  cv_.wait(lk, [&] { return inflight_ == 0; });
}

void RequestLoop::release_exclusive() {
  std::unique_lock<std::mutex> lk(mu_);
  --exclusive_;
  cv_.notify_all();
}

void RequestLoop::wake(void* self) {
  auto* l = static_cast<RequestLoop*>(self);
  { std::lock_guard<std::mutex> g(l->mu_); }
  l->cv_.notify_all();
}

bool RequestLoop::reserve_locked(const std::shared_ptr<Request>& r) {
  const RequestShape sh = request_shape(r->n_points, slot_points_, max_slots_);
  const SlotLayout lay = make_slot(plan_, sh.slot_points);
  const int64_t bytes = lay.bytes * sh.slots;
  const int64_t off = pool_.alloc(bytes);
  if (off < 0) return false;
  r->region = off;
  r->region_bytes = bytes;
  r->layout = lay;
  r->slots.assign((size_t)sh.slots, Slot{});
  char* base = static_cast<char*>(plan_->opts.workspace) + off;
  for (int i = 0; i < sh.slots; ++i) {
    r->slots[i].base = base + (int64_t)i * lay.bytes;
    r->slots[i].stream = streams_[next_stream_++ % streams_.size()];
  }
  r->stats.state = ODF_RUNNING;
  r->stats.t_admit = now();
  peak_resident_ = std::max<int32_t>(peak_resident_, (int32_t)sched_.resident() + 1);
  return true;
}

void RequestLoop::dispatch_locked(std::unique_lock<std::mutex>& lk, const std::shared_ptr<Request>& rp,
                                  int si) {
  Request& r = *rp;
  Slot& s = r.slots[si];
  const int ci = free_ctx_.back();
  free_ctx_.pop_back();
  BatchCtx& c = ctx_[ci];
  const SlotLayout& L = r.layout;
  const int32_t n = std::min(L.points, r.n_points - r.next);
  const int32_t first = r.next;
  const int S = plan_->n_species;
  const int32_t P = slot_points_;
  double* h = c.h_pts;
  std::memcpy(h, r.T.data() + first, 8 * n);
  std::memcpy(h + P, r.logP.data() + first, 8 * n);
  std::memcpy(h + 2 * P, r.vt.data() + first, 8 * n);
  std::memcpy(h + 3 * P, r.abundance.data(), 8 * S);
  r.next += n;
  r.inflight++;
  inflight_++;
  s.busy = true;
  s.failed = false;
  s.ctx = ci;
  s.first = first;
  s.count = n;
  odf_status st = ODF_OK;
  hipError_t e = hipSuccess;
  bool enqueued = false;
  if (r.force_fail) {
    r.force_fail = false;
    set_error("forced failure of a batch launch (test hook)");
    st = ODF_E_DEVICE;
  }
  if (st == ODF_OK) {
    enqueued = true;
    if ((e = hipStreamWaitEvent(s.stream, r.ready, 0)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + L.off_T, h, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + L.off_logP, h + P, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + L.off_vt, h + 2 * P, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + L.off_abund, h + 3 * P, 8 * S, hipMemcpyHostToDevice, s.stream)) != hipSuccess) {
      set_error("request loop copy failed: %s", hipGetErrorString(e));
      st = ODF_E_DEVICE;
    }
  }
  Batch B{};
  if (st == ODF_OK) {
    B = make_batch(plan_, L, s.base, n);
    char* outp = static_cast<char*>(r.out) + (size_t)first * out_point_bytes(plan_);
    st = enqueue_batch(plan_, B, s.base, L, outp, s.stream);
  }
  if (st == ODF_OK) {
    if ((e = hipMemcpyAsync(c.h_nsurv, B.nsurv, 4 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c.h_nsamp, B.nsamp, 8 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(c.h_nit, B.nit, 4 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipEventRecord(c.done, s.stream)) != hipSuccess) {
      set_error("request loop read-back failed: %s", hipGetErrorString(e));
      st = ODF_E_DEVICE;
    }
  }
  if (st == ODF_OK) {
    // wake the loop when the batch is done (a timed wait covers a failure)
    (void)hipLaunchHostFunc(s.stream, &RequestLoop::wake, this);
    return;
  }
  const std::string msg = g_last_error_copy();
  if (!enqueued) {
    finish_locked(rp, s, false, msg.c_str());
    return;
  }
  // part of the batch may be queued and still use the slot and the staging:
  // the slot stays busy until that work has drained
  std::snprintf(s.msg, sizeof s.msg, "%s", msg.c_str());
  s.failed = true;
  if (hipEventRecord(c.done, s.stream) == hipSuccess) {
    (void)hipLaunchHostFunc(s.stream, &RequestLoop::wake, this);
    return;
  }
  lk.unlock();   // queued host functions take the lock
  (void)hipStreamSynchronize(s.stream);
  lk.lock();
  finish_locked(rp, s, false, s.msg);
}

void RequestLoop::finish_locked(const std::shared_ptr<Request>& rp, Slot& s, bool ok, const char* msg) {
  Request& r = *rp;
  BatchCtx& c = ctx_[s.ctx];
  r.inflight--;
  inflight_--;
  if (ok) {
    r.done += s.count;
    for (int i = 0; i < s.count; ++i) {
      r.stats.survivors += c.h_nsurv[i];
      r.stats.voigt_samples += (int64_t)c.h_nsamp[i];
    }
    r.stats.line_evals += (int64_t)s.count * plan_->n_lines;
  } else if (!r.failed) {
    r.failed = true;
    std::snprintf(r.stats.msg, sizeof r.stats.msg, "%s", msg ? msg : "batch failed");
  }
  free_ctx_.push_back(s.ctx);
  s.ctx = -1;
  s.busy = false;
  s.failed = false;
  const bool final_failed = r.failed && r.inflight == 0;
  const bool final_done = !r.failed && r.done == r.n_points;
  if (final_failed || final_done) {
    r.stats.state = final_done ? ODF_DONE : ODF_FAILED;
    r.stats.t_done = now();
    pool_.release(r.region);
    r.region = -1;
    r.slots.clear();
    if (r.ready) (void)hipEventDestroy(r.ready);
    r.ready = nullptr;
    sched_.retire(rp);
  }
  cv_.notify_all();
}

void RequestLoop::run() {
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    bool progress = false;
    const std::vector<std::shared_ptr<Request>> act = sched_.active();
    for (const auto& r : act) {
      for (size_t i = 0; i < r->slots.size(); ++i) {
        Slot& s = r->slots[i];
        if (!s.busy) continue;
        const hipError_t q = hipEventQuery(ctx_[s.ctx].done);
        if (q == hipErrorNotReady) continue;
        progress = true;
        if (q != hipSuccess) {
          finish_locked(r, s, false, hipGetErrorString(q));
        } else if (s.failed) {
          char msg[128];
          std::snprintf(msg, sizeof msg, "%s", s.msg);
          finish_locked(r, s, false, msg);
        } else {
          int bad = -1;
          for (int k = 0; k < s.count && bad < 0; ++k)
            if (ctx_[s.ctx].h_nit[k] < 0) bad = k;
          if (bad < 0) {
            finish_locked(r, s, true, "");
          } else {
            char msg[128];
            std::snprintf(msg, sizeof msg, "ionisation equilibrium did not converge at point %d",
                          s.first + bad);
            finish_locked(r, s, false, msg);
          }
        }
        if (r->slots.empty()) break;   // the request reached its final state
      }
    }
    if (!exclusive_) {
      if (sched_.admit([&](const std::shared_ptr<Request>& r) { return reserve_locked(r); },
                       [&](const std::shared_ptr<Request>& r) {
                         r->stats.state = ODF_DONE;
                         r->stats.t_admit = r->stats.t_done = now();
                         if (r->ready) (void)hipEventDestroy(r->ready);
                         r->ready = nullptr;
                         cv_.notify_all();
                       }))
        progress = true;
      while (!free_ctx_.empty() && !exclusive_) {
        std::shared_ptr<Request> pick =
            sched_.pick([](const std::shared_ptr<Request>& r) { return r->free_slot() >= 0; });
        if (!pick) break;
        dispatch_locked(lk, pick, pick->free_slot());
        progress = true;
      }
    }
    if (stop_ && sched_.idle() && inflight_ == 0) break;
    if (!progress) {
      if (inflight_ > 0)
        cv_.wait_for(lk, std::chrono::milliseconds(20));
      else
        cv_.wait(lk);
    }
  }
}

}  // namespace odf

extern "C" {

odf_status odf_submit(odf_plan_t* plan, const odf_request* req, int64_t* ticket) {
  odf::g_last_error_clear();
  if (!plan) { odf::set_error("plan is NULL"); return ODF_E_INVALID; }
  return plan->loop->submit(req, ticket);
}

odf_status odf_poll(odf_plan_t* plan, int64_t ticket, odf_stats* out) {
  odf::g_last_error_clear();
  if (!plan) { odf::set_error("plan is NULL"); return ODF_E_INVALID; }
  return plan->loop->poll(ticket, out);
}

odf_status odf_wait(odf_plan_t* plan, int64_t ticket, double timeout_s, odf_stats* out) {
  odf::g_last_error_clear();
  if (!plan) { odf::set_error("plan is NULL"); return ODF_E_INVALID; }
  return plan->loop->wait(ticket, timeout_s, out);
}

int64_t odf_request_footprint(const odf_plan_t* plan, int32_t n_points) {
  if (!plan) return -1;
  return plan->loop->footprint(n_points);
}

odf_status odf_loop_status(odf_plan_t* plan, odf_loop_info* out) {
  odf::g_last_error_clear();
  if (!plan || !out) { odf::set_error("odf_loop_status: NULL argument"); return ODF_E_INVALID; }
  plan->loop->info(out);
  return ODF_OK;
}

odf_status odf_debug_fail_next_batch(odf_plan_t* plan, int64_t ticket) {
  odf::g_last_error_clear();
  if (!plan) { odf::set_error("plan is NULL"); return ODF_E_INVALID; }
  return plan->loop->fail_next_batch(ticket);
}

}  // extern "C"

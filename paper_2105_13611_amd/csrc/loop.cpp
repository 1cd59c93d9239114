// Continuous-batching request loop (see loop.h).
#include "loop.h"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace odf {

double RequestLoop::now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

RequestLoop::RequestLoop(odf_plan_s* p) : plan_(p) {
  const int64_t ws = p->opts.workspace_bytes;
  int32_t pts = std::max<int32_t>(1, std::min<int32_t>(p->compute_points, 16));
  layout_ = make_slot(p, pts);
  while (pts > 1 && layout_.bytes * 2 > ws) {  // prefer at least two slots
    pts = std::max(1, pts / 2);
    layout_ = make_slot(p, pts);
  }
  const int64_t n = std::max<int64_t>(1, std::min<int64_t>(ws / layout_.bytes, 32));
  slots_.resize((size_t)n);
  char* base = static_cast<char*>(p->opts.workspace);
  for (int64_t i = 0; i < n; ++i) slots_[i].base = base + i * layout_.bytes;
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
  for (auto& s : slots_) {
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.h_pts) (void)hipHostFree(s.h_pts);
    if (s.h_nsurv) (void)hipHostFree(s.h_nsurv);
    if (s.h_nsamp) (void)hipHostFree(s.h_nsamp);
    if (s.h_nit) (void)hipHostFree(s.h_nit);
  }
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
  const int32_t P = layout_.points, S = plan_->n_species;
  for (size_t i = 0; i < slots_.size(); ++i) {
    Slot& s = slots_[i];
    s.stream = streams_[i % streams_.size()];
    if (hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&s.h_pts, sizeof(double) * (3 * P + S), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_nsurv, sizeof(int32_t) * P, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_nsamp, sizeof(unsigned long long) * P, hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&s.h_nit, sizeof(int32_t) * P, hipHostMallocDefault) != hipSuccess) {
      set_error("request loop: event or pinned-buffer allocation failed");
      start_failed_ = true;
      return false;
    }
  }
  th_ = std::thread([this] { run(); });
  return true;
}

int64_t RequestLoop::footprint(int32_t n_points) const {
  if (n_points <= 0) return 0;
  const int64_t batches = (n_points + layout_.points - 1) / layout_.points;
  return layout_.bytes * std::min<int64_t>(batches, (int64_t)slots_.size());
}

odf_status RequestLoop::submit(const odf_request* r, int64_t* ticket) {
  odf_status st = validate_request(plan_, r, true);
  if (st != ODF_OK) return st;
  if (!ticket) { set_error("ticket is NULL"); return ODF_E_INVALID; }
  if (layout_.bytes > plan_->opts.workspace_bytes) {
    set_error("request needs %lld workspace bytes, plan has %lld", (long long)layout_.bytes,
              (long long)plan_->opts.workspace_bytes);
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
  std::unique_lock<std::mutex> lk(mu_);
  if (stop_) { set_error("plan is being destroyed"); return ODF_E_CANCELLED; }
  if (!start_locked()) return ODF_E_DEVICE;
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

void RequestLoop::acquire_exclusive() {
  std::unique_lock<std::mutex> lk(mu_);
  ++exclusive_;
  cv_.notify_all();
  cv_.wait(lk, [&] {
    for (auto& s : slots_) if (s.busy) return false;
    return true;
  });
}

void RequestLoop::release_exclusive() {
  std::unique_lock<std::mutex> lk(mu_);
  --exclusive_;
  cv_.notify_all();
}

void RequestLoop::dispatch_locked(Slot& s, const std::shared_ptr<Request>& r) {
  const int32_t n = std::min(layout_.points, r->n_points - r->next);
  const int32_t first = r->next;
  const int S = plan_->n_species;
  double* h = s.h_pts;
  std::memcpy(h, r->T.data() + first, 8 * n);
  std::memcpy(h + layout_.points, r->logP.data() + first, 8 * n);
  std::memcpy(h + 2 * layout_.points, r->vt.data() + first, 8 * n);
  std::memcpy(h + 3 * layout_.points, r->abundance.data(), 8 * S);
  if (r->stats.state == ODF_PENDING) {
    r->stats.state = ODF_RUNNING;
    r->stats.t_admit = now();
  }
  r->next += n;
  odf_status st = ODF_OK;
  hipError_t e = hipSuccess;
  if (r->force_fail) {
    r->force_fail = false;
    set_error("forced failure of a batch launch (test hook)");
    st = ODF_E_DEVICE;
  }
  if (st == ODF_OK) {
    if ((e = hipMemcpyAsync(s.base + layout_.off_T, h, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + layout_.off_logP, h + layout_.points, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + layout_.off_vt, h + 2 * layout_.points, 8 * n, hipMemcpyHostToDevice, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.base + layout_.off_abund, h + 3 * layout_.points, 8 * S, hipMemcpyHostToDevice, s.stream)) != hipSuccess) {
      set_error("request loop copy failed: %s", hipGetErrorString(e));
      st = ODF_E_DEVICE;
    }
  }
  Batch B{};
  if (st == ODF_OK) {
    B = make_batch(plan_, layout_, s.base, n);
    char* outp = static_cast<char*>(r->out) + (size_t)first * out_point_bytes(plan_);
    st = enqueue_batch(plan_, B, s.base, layout_, outp, s.stream);
  }
  if (st == ODF_OK) {
    if ((e = hipMemcpyAsync(s.h_nsurv, B.nsurv, 4 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.h_nsamp, B.nsamp, 8 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipMemcpyAsync(s.h_nit, B.nit, 4 * n, hipMemcpyDeviceToHost, s.stream)) != hipSuccess ||
        (e = hipEventRecord(s.done, s.stream)) != hipSuccess) {
      set_error("request loop read-back failed: %s", hipGetErrorString(e));
      st = ODF_E_DEVICE;
    }
  }
  s.req = r;
  s.first = first;
  s.count = n;
  r->inflight++;
  if (st != ODF_OK) {
    s.busy = true;          // finish it at once as failed
    finish_locked(s, false, g_last_error_copy().c_str());
    return;
  }
  s.busy = true;
}

void RequestLoop::finish_locked(Slot& s, bool ok, const char* msg) {
  auto r = s.req;
  r->inflight--;
  if (ok) {
    r->done += s.count;
    for (int i = 0; i < s.count; ++i) {
      r->stats.survivors += s.h_nsurv[i];
      r->stats.voigt_samples += (int64_t)s.h_nsamp[i];
    }
    r->stats.line_evals += (int64_t)s.count * plan_->n_lines;
  } else if (!r->failed) {
    r->failed = true;
    std::snprintf(r->stats.msg, sizeof r->stats.msg, "%s", msg ? msg : "batch failed");
  }
  s.busy = false;
  s.req.reset();
  const bool final_failed = r->failed && r->inflight == 0;
  const bool final_done = !r->failed && r->done == r->n_points;
  if (final_failed || final_done) {
    r->stats.state = final_done ? ODF_DONE : ODF_FAILED;
    r->stats.t_done = now();
    sched_.retire(r);
  }
  cv_.notify_all();
}

void RequestLoop::run() {
  std::unique_lock<std::mutex> lk(mu_);
  while (true) {
    bool progress = false;
    bool any_busy = false;
    for (auto& s : slots_) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipSuccess) {
        int bad = -1;
        for (int i = 0; i < s.count && bad < 0; ++i)
          if (s.h_nit[i] < 0) bad = i;
        if (bad < 0) {
          finish_locked(s, true, "");
        } else {
          char msg[128];
          std::snprintf(msg, sizeof msg, "ionisation equilibrium did not converge at point %d",
                        s.first + bad);
          finish_locked(s, false, msg);
        }
        progress = true;
      } else if (q != hipErrorNotReady) {
        finish_locked(s, false, hipGetErrorString(q));
        progress = true;
      } else {
        any_busy = true;
      }
    }
    if (!exclusive_) {
      if (sched_.admit([&](const std::shared_ptr<Request>& r) {
            r->stats.state = ODF_DONE;
            r->stats.t_admit = r->stats.t_done = now();
            cv_.notify_all();
          }))
        progress = true;
      for (auto& s : slots_) {
        if (s.busy) continue;
        std::shared_ptr<Request> pick = sched_.pick();
        if (!pick) break;
        dispatch_locked(s, pick);
        if (s.busy) any_busy = true;
        progress = true;
      }
    }
    if (stop_ && sched_.idle() && !any_busy) break;
    if (!progress) {
      if (!any_busy) {
        cv_.wait(lk);
      } else {
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(50));
        lk.lock();
      }
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

odf_status odf_debug_fail_next_batch(odf_plan_t* plan, int64_t ticket) {
  odf::g_last_error_clear();
  if (!plan) { odf::set_error("plan is NULL"); return ODF_E_INVALID; }
  return plan->loop->fail_next_batch(ticket);
}

}  // extern "C"

// Admission and batch hand-out policy of the request loop.  It holds no HIP
// state, so the policy runs (and is tested) on the host alone.
//
//   - Requests wait in arrival order and are admitted while fewer than
//     max_active are resident.  A resident request holds no memory of its
//     own: its batches run in the workspace slots.
//   - A request with no points completes at admission.
//   - Each free slot takes one batch from the resident requests in turn,
//     starting after the one served last, and skips failed requests and
//     those whose points have all been handed out.
//
// R must have `int32_t n_points, next` (points handed out so far) and
// `bool failed`.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <memory>
#include <vector>

namespace odf {

template <class R>
class BatchScheduler {
 public:
  explicit BatchScheduler(int32_t max_active) : max_active_(max_active) {}

  void enqueue(std::shared_ptr<R> r) { queue_.push_back(std::move(r)); }

  // Admits waiting requests while there is room; `done_at_once` is called
  // for each one without points.  Returns whether anything was admitted.
  template <class F>
  bool admit(F&& done_at_once) {
    bool any = false;
    while (!queue_.empty() && (int32_t)active_.size() < max_active_) {
      std::shared_ptr<R> r = queue_.front();
      queue_.pop_front();
      any = true;
      if (r->n_points == 0) {
        done_at_once(r);
        continue;
      }
      active_.push_back(std::move(r));
    }
    return any;
  }

  // The request that the next free slot serves, or null.
  std::shared_ptr<R> pick() {
    const size_t n = active_.size();
    for (size_t k = 0; k < n; ++k) {
      const size_t i = (rr_ + k) % n;
      const std::shared_ptr<R>& c = active_[i];
      if (!c->failed && c->next < c->n_points) {
        rr_ = (i + 1) % n;
        return c;
      }
    }
    return nullptr;
  }

  // A request that reached its final state leaves the resident set.
  // The turn stays with the request that was next.
  void retire(const std::shared_ptr<R>& r) {
    const auto it = std::find(active_.begin(), active_.end(), r);
    if (it == active_.end()) return;
    const size_t i = (size_t)(it - active_.begin());
    active_.erase(it);
    if (i < rr_) --rr_;
    if (rr_ >= active_.size()) rr_ = 0;
  }

  bool idle() const { return queue_.empty() && active_.empty(); }
  size_t resident() const { return active_.size(); }
  // Requests not yet admitted (cancelled when the loop stops).
  std::deque<std::shared_ptr<R>>& waiting() { return queue_; }

 private:
  std::deque<std::shared_ptr<R>> queue_;
  std::vector<std::shared_ptr<R>> active_;
  size_t rr_ = 0;
  int32_t max_active_;
};

}  // namespace odf

// Admission and batch hand-out policy of the request loop, and the byte pool
// that admission reserves from.  No HIP state, so the policy runs (and is
// tested) on the host alone.
//
//   - The workspace is a pool of bytes.  A request reserves its footprint
//     (its own batch slots) from the pool when it is admitted and releases
//     it when it reaches a final state.
//   - Requests are admitted in arrival order while the first waiting one
//     fits the free bytes; a later, smaller request never overtakes it.
//   - A request with no points completes at admission and takes nothing.
//   - Each dispatch takes one batch from the resident requests in turn,
//     starting after the one served last, skipping failed requests, those
//     whose points have all been handed out and those the caller's
//     predicate rejects (no free slot of their own).
//
// R must have `int32_t n_points, next` (points handed out so far) and
// `bool failed`.
#pragma once

#include <algorithm>
#include <cstddef>
#include <cstdint>
#include <deque>
#include <iterator>
#include <map>
#include <memory>
#include <vector>

namespace odf {

// First-fit allocator over [0, capacity) with aligned block sizes.  Freed
// blocks merge with free neighbours, so the pool returns to one block when
// everything is released.
class BytePool {
 public:
  explicit BytePool(int64_t capacity = 0, int64_t align = 256) { reset(capacity, align); }

  void reset(int64_t capacity, int64_t align = 256) {
    align_ = std::max<int64_t>(align, 1);
    cap_ = capacity / align_ * align_;
    free_.clear();
    used_blocks_.clear();
    if (cap_ > 0) free_[0] = cap_;
    used_ = peak_ = 0;
  }

  // Offset of a block of at least `bytes`, or -1 when no free block holds it.
  int64_t alloc(int64_t bytes) {
    if (bytes <= 0) return -1;
    const int64_t need = (bytes + align_ - 1) / align_ * align_;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const int64_t off = it->first, rest = it->second - need;
      free_.erase(it);
      if (rest > 0) free_[off + need] = rest;
      used_blocks_[off] = need;
      used_ += need;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return -1;
  }

  // Returns a block from alloc(); unknown offsets are ignored.
  void release(int64_t off) {
    auto u = used_blocks_.find(off);
    if (u == used_blocks_.end()) return;
    int64_t start = off, size = u->second;
    used_ -= size;
    used_blocks_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + size) {
      size += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        size += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = size;
  }

  int64_t capacity() const { return cap_; }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }
  int64_t largest_free() const {
    int64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  size_t free_blocks() const { return free_.size(); }

 private:
  int64_t align_ = 256, cap_ = 0, used_ = 0, peak_ = 0;
  std::map<int64_t, int64_t> free_;        // offset -> size
  std::map<int64_t, int64_t> used_blocks_; // offset -> size
};

// Batch slots a request of n points reserves: slots of min(n, slot_points)
// points, as many as its batches up to max_slots (at least one).
struct RequestShape {
  int32_t slot_points = 0;
  int32_t slots = 0;
};
inline RequestShape request_shape(int32_t n_points, int32_t slot_points, int32_t max_slots) {
  RequestShape s;
  if (n_points <= 0) return s;
  s.slot_points = std::min(n_points, std::max(slot_points, 1));
  const int32_t batches = (n_points + s.slot_points - 1) / s.slot_points;
  s.slots = std::max(1, std::min(batches, max_slots));
  return s;
}

template <class R>
class BatchScheduler {
 public:
  BatchScheduler() = default;

  void enqueue(std::shared_ptr<R> r) { queue_.push_back(std::move(r)); }

  // Admits waiting requests in arrival order while `reserve(r)` succeeds
  // (it reserves the request's footprint and returns false when that does
  // not fit now); `done_at_once(r)` is called for each request without
  // points instead.  Returns whether anything was admitted.
  template <class Reserve, class Done>
  bool admit(Reserve&& reserve, Done&& done_at_once) {
    bool any = false;
    while (!queue_.empty()) {
      std::shared_ptr<R> r = queue_.front();
      if (r->n_points == 0) {
        queue_.pop_front();
        done_at_once(r);
        any = true;
        continue;
      }
      if (!reserve(r)) break;
      queue_.pop_front();
      active_.push_back(std::move(r));
      any = true;
    }
    return any;
  }

  // The request that the next dispatch serves, or null.
  template <class Pred>
  std::shared_ptr<R> pick(Pred&& ready) {
    const size_t n = active_.size();
    for (size_t k = 0; k < n; ++k) {
      const size_t i = (rr_ + k) % n;
      const std::shared_ptr<R>& c = active_[i];
      if (!c->failed && c->next < c->n_points && ready(c)) {
        rr_ = (i + 1) % n;
        return c;
      }
    }
    return nullptr;
  }
  std::shared_ptr<R> pick() {
    return pick([](const std::shared_ptr<R>&) { return true; });
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
  const std::vector<std::shared_ptr<R>>& active() const { return active_; }
  // Requests not yet admitted (cancelled when the loop stops).
  std::deque<std::shared_ptr<R>>& waiting() { return queue_; }

 private:
  std::deque<std::shared_ptr<R>> queue_;
  std::vector<std::shared_ptr<R>> active_;
  size_t rr_ = 0;
};

}  // namespace odf

// Host-only test of the request loop's admission and batch hand-out policy
// and of the byte pool admission reserves from
// (paper_2105_13611_amd/csrc/scheduler.h).  Prints "ok" and exits 0, or
// names the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <vector>

#include "scheduler.h"

struct Req {
  int id;
  int32_t n_points, next = 0;
  bool failed = false;
  int64_t bytes = 0;      // footprint
  int64_t off = -1;       // reserved block
  int slots = 1, busy = 0;
  Req(int i, int32_t n, int64_t b = 0) : id(i), n_points(n), bytes(b) {}
};
using P = std::shared_ptr<Req>;

static int fails = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAILED line %d: %s\n", __LINE__, #c);           \
      ++fails;                                                     \
    }                                                              \
  } while (0)

// hands out one batch of `b` points of the picked request; returns its id or -1
static int serve(odf::BatchScheduler<Req>& s, int32_t b) {
  P r = s.pick();
  if (!r) return -1;
  r->next += std::min(b, r->n_points - r->next);
  return r->id;
}

// admission that reserves each request's footprint from `pool`
static bool admit(odf::BatchScheduler<Req>& s, odf::BytePool& pool, std::vector<int>* done = nullptr) {
  return s.admit(
      [&](const P& q) {
        q->off = pool.alloc(q->bytes);
        return q->off >= 0;
      },
      [&](const P& q) {
        if (done) done->push_back(q->id);
      });
}

static void retire(odf::BatchScheduler<Req>& s, odf::BytePool& pool, const P& r) {
  pool.release(r->off);
  r->off = -1;
  s.retire(r);
}

int main() {
  {  // byte pool: first fit, alignment, merging of freed neighbours, peak
    odf::BytePool p(10 * 256 + 100, 256);
    CHECK(p.capacity() == 10 * 256);
    const int64_t a = p.alloc(300), b = p.alloc(256), c = p.alloc(1);
    CHECK(a == 0 && b == 512 && c == 768);
    CHECK(p.used() == 3 * 256 + 256 && p.peak() == 1024);
    CHECK(p.alloc(7 * 256) == -1);              // 6 blocks of 256 left
    const int64_t d = p.alloc(6 * 256);
    CHECK(d == 1024 && p.largest_free() == 0);
    p.release(b);
    CHECK(p.alloc(512) == -1);                  // one 256 hole only
    CHECK(p.alloc(256) == 512);
    p.release(512);
    p.release(a);                               // 0..768 free, merged
    CHECK(p.largest_free() == 768 && p.free_blocks() == 1);
    CHECK(p.alloc(700) == 0);
    p.release(0);
    p.release(c);
    p.release(d);
    CHECK(p.used() == 0 && p.free_blocks() == 1 && p.largest_free() == p.capacity());
    CHECK(p.peak() == 10 * 256);
    p.release(12345);                           // unknown: ignored
    CHECK(p.alloc(0) == -1 && p.alloc(p.capacity() + 1) == -1);
  }
  {  // request shapes: slots of min(n, slot_points) points, up to max_slots
    const odf::RequestShape s0 = odf::request_shape(0, 16, 2), s1 = odf::request_shape(1, 16, 2),
                            s16 = odf::request_shape(16, 16, 2), s17 = odf::request_shape(17, 16, 2),
                            s1000 = odf::request_shape(1000, 16, 2), s5 = odf::request_shape(5, 16, 1);
    CHECK(s0.slots == 0);
    CHECK(s1.slot_points == 1 && s1.slots == 1);
    CHECK(s16.slot_points == 16 && s16.slots == 1);
    CHECK(s17.slot_points == 16 && s17.slots == 2);
    CHECK(s1000.slot_points == 16 && s1000.slots == 2);
    CHECK(s5.slot_points == 5 && s5.slots == 1);
  }
  {  // admission by footprint, in arrival order: a large head waits for room
     // and later small requests do not overtake it
    odf::BytePool pool(100 * 256, 256);
    odf::BatchScheduler<Req> s;
    P a = std::make_shared<Req>(0, 8, 60 * 256), b = std::make_shared<Req>(1, 8, 30 * 256),
      c = std::make_shared<Req>(2, 8, 50 * 256), d = std::make_shared<Req>(3, 8, 5 * 256);
    for (const P& r : {a, b, c, d}) s.enqueue(r);
    CHECK(admit(s, pool));
    CHECK(s.resident() == 2 && pool.used() == 90 * 256);   // c does not fit; d waits behind it
    CHECK(!admit(s, pool));
    retire(s, pool, b);
    CHECK(!admit(s, pool) && s.resident() == 1);            // 40 free: c still waits
    retire(s, pool, a);
    CHECK(admit(s, pool) && s.resident() == 2 && pool.used() == 55 * 256);
    retire(s, pool, c);
    retire(s, pool, d);
    CHECK(s.idle() && pool.used() == 0 && pool.peak() == 90 * 256);
  }
  {  // requests without points complete at admission and take nothing
    odf::BytePool pool(10 * 256, 256);
    odf::BatchScheduler<Req> s;
    P a = std::make_shared<Req>(0, 0), b = std::make_shared<Req>(1, 0), c = std::make_shared<Req>(2, 3, 256);
    s.enqueue(a);
    s.enqueue(b);
    s.enqueue(c);
    std::vector<int> done;
    admit(s, pool, &done);
    CHECK(done.size() == 2 && done[0] == 0 && done[1] == 1);
    CHECK(s.resident() == 1 && pool.used() == 256);
    CHECK(serve(s, 2) == 2 && serve(s, 2) == 2 && serve(s, 2) == -1);
  }
  {  // round robin over the resident ones; failed requests are skipped
    odf::BytePool pool(1000 * 256, 256);
    odf::BatchScheduler<Req> s;
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 100, 256));
      s.enqueue(r.back());
    }
    admit(s, pool);
    CHECK(serve(s, 1) == 0);
    r[1]->failed = true;
    CHECK(serve(s, 1) == 2);
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 2);
    retire(s, pool, r[1]);           // the failed one leaves once final
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 2);
    retire(s, pool, r[0]);
    CHECK(serve(s, 1) == 2 && serve(s, 1) == 2);
  }
  {  // the predicate: a request without a free slot of its own is passed over
    odf::BytePool pool(1000 * 256, 256);
    odf::BatchScheduler<Req> s;
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 100, 256));
      s.enqueue(r.back());
    }
    admit(s, pool);
    auto ready = [](const P& q) { return q->busy < q->slots; };
    P x = s.pick(ready);
    CHECK(x && x->id == 0);
    x->busy = 1;
    x = s.pick(ready);
    CHECK(x && x->id == 1);
    x->busy = 1;
    x = s.pick(ready);
    CHECK(x && x->id == 2);
    x->busy = 1;
    CHECK(!s.pick(ready));
    r[1]->busy = 0;
    x = s.pick(ready);
    CHECK(x && x->id == 1);
  }
  {  // retiring a request served earlier keeps the turn with the next one
    odf::BytePool pool(1000 * 256, 256);
    odf::BatchScheduler<Req> s;
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 100, 256));
      s.enqueue(r.back());
    }
    admit(s, pool);
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 1);
    retire(s, pool, r[0]);           // request 2 was next
    CHECK(serve(s, 1) == 2);
    CHECK(serve(s, 1) == 1);
    retire(s, pool, r[2]);           // retiring the one just served
    CHECK(serve(s, 1) == 1);
    s.retire(r[0]);                  // not resident: no effect
    CHECK(s.resident() == 1);
  }
  {  // fairness: three long requests share the batches evenly
    odf::BytePool pool(1000 * 256, 256);
    odf::BatchScheduler<Req> s;
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 1000, 256));
      s.enqueue(r.back());
    }
    admit(s, pool);
    int count[3] = {0, 0, 0};
    for (int k = 0; k < 300; ++k) ++count[serve(s, 1)];
    CHECK(count[0] == 100 && count[1] == 100 && count[2] == 100);
  }
  {  // a random stream: the reserved bytes never exceed the pool and equal
     // the resident requests' footprints; admission keeps arrival order and
     // every request is admitted and completes
    std::mt19937 rng(7);
    odf::BytePool pool(64 * 256, 256);
    odf::BatchScheduler<Req> s;
    std::vector<P> all;
    int next_admit = 0, completed = 0;
    for (int step = 0; step < 4000; ++step) {
      if (all.size() < 300 && rng() % 3 == 0) {
        const int64_t units = 1 + rng() % 40;
        all.push_back(std::make_shared<Req>((int)all.size(), 1 + rng() % 50, units * 256));
        s.enqueue(all.back());
      }
      std::vector<int> done;
      admit(s, pool, &done);
      for (const P& q : s.active()) {
        if (q->id >= next_admit) {
          CHECK(q->id == next_admit);    // in arrival order
          next_admit = q->id + 1;
        }
      }
      int64_t sum = 0;
      for (const P& q : s.active()) sum += q->bytes;
      CHECK(sum == pool.used() && pool.used() <= pool.capacity());
      if (serve(s, 8) < 0 && !s.active().empty()) {
        // every point handed out: the oldest resident one completes
        std::vector<P> act = s.active();
        for (const P& q : act)
          if (q->next == q->n_points) {
            retire(s, pool, q);
            ++completed;
            break;
          }
      }
    }
    while (!s.idle()) {
      admit(s, pool);
      while (serve(s, 8) >= 0) {
      }
      std::vector<P> act = s.active();
      for (const P& q : act) {
        retire(s, pool, q);
        ++completed;
      }
    }
    CHECK(completed == (int)all.size() && pool.used() == 0 && pool.free_blocks() == 1);
    CHECK(pool.peak() <= pool.capacity());
  }
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}

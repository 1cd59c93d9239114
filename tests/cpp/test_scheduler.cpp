// Host-only test of the request loop's admission and batch hand-out policy
// (paper_2105_13611_amd/csrc/scheduler.h).  Prints "ok" and exits 0, or
// names the failed check and exits 1.
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#include "scheduler.h"

struct Req {
  int id;
  int32_t n_points, next = 0;
  bool failed = false;
  Req(int i, int32_t n) : id(i), n_points(n) {}
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

int main() {
  {  // admission in arrival order, at most max_active resident
    odf::BatchScheduler<Req> s(2);
    std::vector<P> r;
    for (int i = 0; i < 4; ++i) {
      r.push_back(std::make_shared<Req>(i, 8));
      s.enqueue(r.back());
    }
    std::vector<int> empty;
    CHECK(s.admit([&](const P& q) { empty.push_back(q->id); }));
    CHECK(s.resident() == 2 && empty.empty());
    // round-robin over the resident ones: 0 1 0 1 ...
    CHECK(serve(s, 4) == 0);
    CHECK(serve(s, 4) == 1);
    CHECK(serve(s, 4) == 0);
    CHECK(serve(s, 4) == 1);
    CHECK(serve(s, 4) == -1);        // every point handed out
    s.retire(r[0]);
    CHECK(s.admit([&](const P&) {}));
    CHECK(s.resident() == 2);        // request 2 took the free place
    CHECK(serve(s, 4) == 2);
    CHECK(!s.admit([&](const P&) {}));   // still full
    s.retire(r[1]);
    s.retire(r[2]);
    CHECK(s.admit([&](const P&) {}));
    CHECK(serve(s, 8) == 3);
    s.retire(r[3]);
    CHECK(s.idle());
  }
  {  // requests without points complete at admission and take no place
    odf::BatchScheduler<Req> s(1);
    P a = std::make_shared<Req>(0, 0), b = std::make_shared<Req>(1, 0), c = std::make_shared<Req>(2, 3);
    s.enqueue(a);
    s.enqueue(b);
    s.enqueue(c);
    std::vector<int> done;
    s.admit([&](const P& q) { done.push_back(q->id); });
    CHECK(done.size() == 2 && done[0] == 0 && done[1] == 1);
    CHECK(s.resident() == 1);
    CHECK(serve(s, 2) == 2 && serve(s, 2) == 2 && serve(s, 2) == -1);
  }
  {  // failed requests are skipped; the turn continues after the last served
    odf::BatchScheduler<Req> s(3);
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 100));
      s.enqueue(r.back());
    }
    s.admit([&](const P&) {});
    CHECK(serve(s, 1) == 0);
    r[1]->failed = true;
    CHECK(serve(s, 1) == 2);
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 2);
    s.retire(r[1]);                  // the failed one leaves once final
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 2);
    s.retire(r[0]);
    CHECK(serve(s, 1) == 2 && serve(s, 1) == 2);
  }
  {  // retiring a request served earlier keeps the turn with the next one
    odf::BatchScheduler<Req> s(4);
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 100));
      s.enqueue(r.back());
    }
    s.admit([&](const P&) {});
    CHECK(serve(s, 1) == 0);
    CHECK(serve(s, 1) == 1);
    s.retire(r[0]);                  // request 2 was next
    CHECK(serve(s, 1) == 2);
    CHECK(serve(s, 1) == 1);
    s.retire(r[2]);                  // retiring the one just served
    CHECK(serve(s, 1) == 1);
    s.retire(r[0]);                  // not resident: no effect
    CHECK(s.resident() == 1);
  }
  {  // fairness: three long requests share the slots evenly
    odf::BatchScheduler<Req> s(16);
    std::vector<P> r;
    for (int i = 0; i < 3; ++i) {
      r.push_back(std::make_shared<Req>(i, 1000));
      s.enqueue(r.back());
    }
    s.admit([&](const P&) {});
    int count[3] = {0, 0, 0};
    for (int k = 0; k < 300; ++k) ++count[serve(s, 1)];
    CHECK(count[0] == 100 && count[1] == 100 && count[2] == 100);
  }
  if (fails) return 1;
  std::printf("ok\n");
  return 0;
}

// Host-only checks of the projection server's admission scheduler (no GPU).
// Built and run by tests/test_serve_sched_cpu.py with g++.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "serve_sched.h"

using prism::serve::Pick;
using prism::serve::Pool;
using prism::serve::Scheduler;

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
      ++failures;                                                  \
    }                                                              \
  } while (0)

static void pool_basics() {
  Pool p(4096);
  size_t a, b, c, d;
  CHECK(p.alloc(100, &a) && a == 0);
  CHECK(p.alloc(256, &b) && b == 256);
  CHECK(p.alloc(3000, &c) && c == 512);
  CHECK(!p.alloc(1024, &d));                 // 512 + 3072 = 3584 used, 512 left
  CHECK(p.used() == 3584);
  p.release(b, 256);
  CHECK(p.largest_free() == 512);
  p.release(a, 100);                         // coalesces with b's hole
  CHECK(p.free_blocks() == 2);
  p.release(c, 3000);                        // everything free, one block
  CHECK(p.free_blocks() == 1 && p.used() == 0 && p.largest_free() == 4096);
}

static void pool_random_never_overlaps() {
  std::mt19937 rng(7);
  Pool p(1 << 20);
  struct A { size_t off, n; };
  std::vector<A> live;
  for (int step = 0; step < 20000; ++step) {
    if (live.empty() || rng() % 3 != 0) {
      size_t n = 1 + rng() % 50000, off;
      if (p.alloc(n, &off)) {
        const size_t end = off + Pool::round_up(n);
        CHECK(end <= p.capacity());
        for (const A& x : live) CHECK(end <= x.off || x.off + Pool::round_up(x.n) <= off);
        live.push_back({off, n});
      }
    } else {
      const size_t i = rng() % live.size();
      p.release(live[i].off, live[i].n);
      live.erase(live.begin() + i);
    }
    size_t used = 0;
    for (const A& x : live) used += Pool::round_up(x.n);
    if (used != p.used()) { CHECK(used == p.used()); break; }
  }
}

static void fifo_and_controller_serialisation() {
  Scheduler s(1 << 20, 8, 100);
  const int c0 = s.add_controller(1000, 10), c1 = s.add_controller(1000, 10);
  CHECK(c0 == 0 && c1 == 1);
  CHECK(s.submit(c0, 1, 10) == prism::serve::kQueued);
  CHECK(s.submit(c0, 2, 10) == prism::serve::kQueued);   // waits for ticket 1
  CHECK(s.submit(c1, 3, 10) == prism::serve::kQueued);
  std::vector<Pick> p = s.pick();
  CHECK(p.size() == 2 && p[0].ticket == 1 && p[1].ticket == 3);
  CHECK(!p[0].warm && !p[1].warm);                       // first solves start cold
  CHECK(s.pick().empty());                               // ticket 2's controller is busy
  s.complete(c0, true);
  p = s.pick();
  CHECK(p.size() == 1 && p[0].ticket == 2 && p[0].warm); // warm from ticket 1
  s.complete(c0, false);                                 // a failed solve leaves no state
  CHECK(s.submit(c0, 4, 10) == prism::serve::kQueued);
  p = s.pick();
  CHECK(p.size() == 1 && !p[0].warm);
  s.complete(c0, true);
  CHECK(s.submit(c0, 5, 7) == prism::serve::kQueued);    // different sample count: cold
  p = s.pick();
  CHECK(p.size() == 1 && !p[0].warm);
}

static void eviction_lru_and_blocking() {
  // room for two states of 1000 bytes (1024 after rounding)
  Scheduler s(2048, 8, 100);
  const int a = s.add_controller(1000, 1), b = s.add_controller(1000, 1), c = s.add_controller(1000, 1);
  CHECK(s.add_controller(5000, 1) == -1);                // larger than the budget
  s.submit(a, 1, 1);
  s.submit(b, 2, 1);
  std::vector<Pick> p = s.pick();
  CHECK(p.size() == 2);
  s.submit(c, 3, 1);
  CHECK(s.pick().empty());                               // a, b busy: nothing to evict
  s.complete(b, true);
  s.complete(a, true);                                   // a used last... by clock, a picked first
  p = s.pick();
  CHECK(p.size() == 1 && p[0].ticket == 3 && !p[0].warm);
  CHECK(s.evictions() == 1);
  CHECK(!s.controller(a).resident && s.controller(b).resident);   // a was least recently used
  s.complete(c, true);
  s.submit(a, 4, 1);                                     // a was evicted: starts cold
  p = s.pick();
  CHECK(p.size() == 1 && !p[0].warm);
  CHECK(s.pool().used() <= s.pool().capacity());
}

static void head_of_line_and_max_batch() {
  Scheduler s(4096, 2, 100);
  const int big = s.add_controller(4000, 1), small1 = s.add_controller(100, 1),
            small2 = s.add_controller(100, 1), small3 = s.add_controller(100, 1);
  s.submit(small1, 1, 1);
  CHECK(s.pick().size() == 1);                           // small1 resident and busy
  s.submit(big, 2, 1);                                   // cannot be placed while small1 runs
  s.submit(small2, 3, 1);
  CHECK(s.pick().empty());                               // FIFO: small2 waits behind big
  s.complete(small1, true);
  std::vector<Pick> p = s.pick();                        // small1 evicted, big placed
  CHECK(p.size() == 1 && p[0].ticket == 2);
  s.complete(big, true);
  s.submit(small3, 4, 1);
  p = s.pick();                                          // evict big; then small2, small3 (cap 2)
  CHECK(p.size() == 2 && p[0].ticket == 3 && p[1].ticket == 4);
}

static void queue_limit() {
  Scheduler s(4096, 4, 2);
  const int a = s.add_controller(100, 1);
  CHECK(s.submit(a, 1, 1) == prism::serve::kQueued);
  CHECK(s.submit(a, 2, 1) == prism::serve::kQueued);
  CHECK(s.submit(a, 3, 1) == prism::serve::kQueueFull);
  CHECK(s.submit(9, 4, 1) == prism::serve::kBadController);
}

static void random_workload_invariants() {
  std::mt19937 rng(11);
  Scheduler s(64 * 1024, 6, 1000);
  std::vector<int> ids;
  for (int i = 0; i < 24; ++i) ids.push_back(s.add_controller(1000 + rng() % 9000, 4));
  std::vector<Pick> running;
  std::set<int64_t> done;
  int64_t next = 1, submitted = 0;
  for (int step = 0; step < 5000; ++step) {
    if (rng() % 2) {
      if (s.submit(ids[rng() % ids.size()], next, 4) == prism::serve::kQueued) ++submitted;
      ++next;
    }
    if (!running.empty() && rng() % 2) {
      const size_t i = rng() % running.size();
      s.complete(running[i].ctrl, true);
      done.insert(running[i].ticket);
      running.erase(running.begin() + i);
    }
    for (const Pick& p : s.pick()) {
      for (const Pick& r : running) CHECK(r.ctrl != p.ctrl);   // one request per controller
      running.push_back(p);
    }
    CHECK(s.pool().used() <= s.pool().capacity());
    // every busy controller is resident and states of resident controllers do not overlap
    for (int i = 0; i < s.controllers(); ++i) {
      const auto& ci = s.controller(i);
      if (ci.busy) CHECK(ci.resident);
      if (!ci.resident) continue;
      for (int k = i + 1; k < s.controllers(); ++k) {
        const auto& ck = s.controller(k);
        if (!ck.resident) continue;
        const size_t ei = ci.off + Pool::round_up(ci.state_bytes), ek = ck.off + Pool::round_up(ck.state_bytes);
        CHECK(ei <= ck.off || ek <= ci.off);
      }
    }
  }
  while (!running.empty() || s.queued() > 0) {             // drain
    for (const Pick& r : running) {
      s.complete(r.ctrl, true);
      done.insert(r.ticket);
    }
    running = s.pick();
  }
  CHECK((int64_t)done.size() == submitted);
}

int main() {
  pool_basics();
  pool_random_never_overlaps();
  fifo_and_controller_serialisation();
  eviction_lru_and_blocking();
  head_of_line_and_max_batch();
  queue_limit();
  random_workload_invariants();
  if (failures) {
    std::printf("%d failures\n", failures);
    return 1;
  }
  std::printf("scheduler: all checks passed\n");
  return 0;
}

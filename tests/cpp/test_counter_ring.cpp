// Host-only check of the tile-queue counter ring (no GPU): a discrete-event model of
// streams and launches in which every launch follows the library's rule (take a set,
// wait on its own stream for the set's previous launch if the ring says so, run,
// record). Checked: no two launches ever hold one set at overlapping times, for any
// number of launches in flight, streams, ring wrap-arounds and durations; the ring
// hands out sets in turn; the first use of a set needs no wait.
// Built and run by tests/test_counter_ring_cpu.py with g++.
#include <algorithm>
#include <cstdio>
#include <random>
#include <vector>

#include "counter_ring.h"

static int failures = 0;
#define CHECK(c)                                                   \
  do {                                                             \
    if (!(c)) {                                                    \
      std::printf("FAIL %s:%d: %s\n", __FILE__, __LINE__, #c);     \
      ++failures;                                                  \
    }                                                              \
  } while (0)

struct Interval {
  double start, end;
};

template <int N>
static void simulate(int n_streams, int n_launches, unsigned seed, bool honour_wait) {
  prism::CounterRing<N> ring;
  std::mt19937 rng(seed);
  std::uniform_int_distribution<int> pick(0, n_streams - 1);
  std::exponential_distribution<double> dur(1.0);
  std::vector<double> stream_free(n_streams, 0.0);   // end of the last launch per stream
  std::vector<double> slot_done(N, 0.0);             // completion of each set's last launch
  std::vector<std::vector<Interval>> held(N);
  int waits = 0;
  for (int i = 0; i < n_launches; ++i) {
    const int s = pick(rng);
    const auto t = ring.take();
    CHECK(t.slot == i % N);                       // in turn
    CHECK(t.wait == (i >= N));                    // every set is used once before a wait
    double start = stream_free[s];
    if (t.wait && honour_wait) {
      start = std::max(start, slot_done[t.slot]);
      ++waits;
    }
    const double end = start + dur(rng) * (1 + (i % 7));
    held[t.slot].push_back({start, end});
    stream_free[s] = end;
    slot_done[t.slot] = end;
    ring.recorded(t.slot);
  }
  int overlaps = 0;
  for (auto& h : held) {
    std::sort(h.begin(), h.end(), [](const Interval& a, const Interval& b) { return a.start < b.start; });
    for (size_t k = 1; k < h.size(); ++k)
      if (h[k].start < h[k - 1].end) ++overlaps;
  }
  if (honour_wait) CHECK(overlaps == 0);
  else CHECK(overlaps > 0);                       // the check is not vacuous
  std::printf("N=%d streams=%d launches=%d wait=%d: %d waits, %d overlaps\n", N, n_streams,
              n_launches, honour_wait ? 1 : 0, waits, overlaps);
}

int main() {
  simulate<64>(1, 1000, 1, true);
  simulate<64>(4, 5000, 2, true);
  simulate<64>(32, 20000, 3, true);
  simulate<4>(16, 5000, 4, true);
  simulate<1>(8, 2000, 5, true);
  simulate<64>(32, 20000, 6, false);      // without the wait, sets collide
  if (failures) {
    std::printf("%d failure(s)\n", failures);
    return 1;
  }
  std::printf("counter ring: all checks passed\n");
  return 0;
}

// Admission scheduler of the projection server: plain C++ (no HIP), so its
// policy can be tested on a host without a GPU.
//
// * Pool: first-fit allocator over one device allocation of `budget` bytes
//   (offsets only; 256-byte granules, neighbours coalesce on free).
// * Each controller's warm state (its last projected trajectories and dual
//   state) lives in the pool while resident. A request is admitted when its
//   controller has nothing in flight and its state is resident or can be made
//   resident, evicting the states of idle controllers least recently used
//   first (an evicted controller's next request starts cold).
// * Admission is first come, first served: the scan stops at the first request
//   whose state cannot be placed, so a large request is never overtaken
//   indefinitely; requests whose controller is busy wait for their own
//   predecessor and do not block others.
#pragma once

#include <cstddef>
#include <cstdint>
#include <deque>
#include <map>
#include <vector>

namespace prism {
namespace serve {

constexpr size_t kGranule = 256;

class Pool {
 public:
  explicit Pool(size_t bytes) : cap_(bytes / kGranule * kGranule) {
    if (cap_ > 0) free_[0] = cap_;
  }
  static size_t round_up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }
  bool alloc(size_t bytes, size_t* off) {
    const size_t need = round_up(bytes == 0 ? 1 : bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      *off = it->first;
      const size_t rest = it->second - need;
      const size_t at = it->first + need;
      free_.erase(it);
      if (rest > 0) free_[at] = rest;
      used_ += need;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    const size_t n = round_up(bytes == 0 ? 1 : bytes);
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t capacity() const { return cap_; }
  size_t used() const { return used_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = f.second > m ? f.second : m;
    return m;
  }
  size_t free_blocks() const { return free_.size(); }

 private:
  size_t cap_;
  size_t used_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
};

struct Controller {
  size_t state_bytes = 0;    // resident footprint
  int max_N = 0;
  bool resident = false;
  size_t off = 0;
  bool busy = false;         // a request is in flight
  bool valid = false;        // the resident state holds a finished solve
  int last_N = -1;           // sample count of that solve
  uint64_t last_use = 0;
};

struct Pick {
  int64_t ticket;
  int ctrl;
  size_t state_off;
  bool warm;                 // start from the resident state of the previous solve
};

enum SubmitResult { kQueued = 0, kQueueFull = 1, kNeverFits = 2, kBadController = 3 };

class Scheduler {
 public:
  Scheduler(size_t budget, int max_batch, size_t max_queue)
      : pool_(budget), max_batch_(max_batch < 1 ? 1 : max_batch), max_queue_(max_queue) {}

  // Returns the controller id, or -1 if its state could never fit the budget.
  int add_controller(size_t state_bytes, int max_N) {
    if (Pool::round_up(state_bytes) > pool_.capacity()) return -1;
    Controller c;
    c.state_bytes = state_bytes;
    c.max_N = max_N;
    ctrls_.push_back(c);
    return (int)ctrls_.size() - 1;
  }

  SubmitResult submit(int ctrl, int64_t ticket, int N) {
    if (ctrl < 0 || ctrl >= (int)ctrls_.size()) return kBadController;
    if (queue_.size() >= max_queue_) return kQueueFull;
    queue_.push_back(Queued{ticket, ctrl, N});
    return kQueued;
  }

  // Requests to launch now (at most max_batch), in arrival order.
  std::vector<Pick> pick() {
    std::vector<Pick> out;
    std::vector<bool> in_pick(ctrls_.size(), false);
    for (auto it = queue_.begin(); it != queue_.end() && (int)out.size() < max_batch_;) {
      Controller& c = ctrls_[it->ctrl];
      if (c.busy || in_pick[it->ctrl]) {
        ++it;
        continue;
      }
      if (!c.resident && !place(it->ctrl, in_pick)) break;
      c.busy = true;
      c.last_use = ++clock_;
      in_pick[it->ctrl] = true;
      const bool warm = c.valid && c.last_N == it->N;
      out.push_back(Pick{it->ticket, it->ctrl, c.off, warm});
      c.last_N = it->N;
      c.valid = false;         // rewritten by this solve
      it = queue_.erase(it);
    }
    return out;
  }

  // The controller's in-flight request ended; ok = its state now holds the solve.
  void complete(int ctrl, bool ok) {
    Controller& c = ctrls_[ctrl];
    c.busy = false;
    c.valid = ok;
  }

  size_t queued() const { return queue_.size(); }
  const Pool& pool() const { return pool_; }
  const Controller& controller(int i) const { return ctrls_[i]; }
  int controllers() const { return (int)ctrls_.size(); }
  uint64_t evictions() const { return evictions_; }

 private:
  struct Queued {
    int64_t ticket;
    int ctrl;
    int N;
  };

  bool place(int ctrl, const std::vector<bool>& in_pick) {
    Controller& c = ctrls_[ctrl];
    size_t off = 0;
    while (!pool_.alloc(c.state_bytes, &off)) {
      int victim = -1;
      for (int i = 0; i < (int)ctrls_.size(); ++i) {
        const Controller& v = ctrls_[i];
        if (!v.resident || v.busy || in_pick[i]) continue;
        if (victim < 0 || v.last_use < ctrls_[victim].last_use) victim = i;
      }
      if (victim < 0) return false;
      Controller& v = ctrls_[victim];
      pool_.release(v.off, v.state_bytes);
      v.resident = false;
      v.valid = false;
      ++evictions_;
    }
    c.resident = true;
    c.off = off;
    c.valid = false;
    return true;
  }

  Pool pool_;
  int max_batch_;
  size_t max_queue_;
  std::vector<Controller> ctrls_;
  std::deque<Queued> queue_;
  uint64_t clock_ = 0;
  uint64_t evictions_ = 0;
};

}  // namespace serve
}  // namespace prism

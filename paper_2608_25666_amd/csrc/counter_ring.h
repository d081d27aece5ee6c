// Reuse order of a handle's tile-queue counter sets (host code, no HIP calls).
//
// A solve launch takes the next set in turn. The launch that used the set before
// may still be running on another stream, so the taker first makes its own stream
// wait for that launch's completion event, then records its own completion on the
// set. Two launches therefore never use one set at the same time, whatever the
// streams, the number of solves in flight, or the order of completions. The caller
// holds a mutex around take() and recorded() (with the launch between them).
#pragma once

namespace prism {

template <int N>
class CounterRing {
 public:
  struct Take {
    int slot;     // counter set to use
    bool wait;    // wait for the completion event of the set's previous launch first
  };
  Take take() {
    const int s = (int)(next_++ % (unsigned)N);
    return {s, used_[s]};
  }
  // The launch on `slot` has been enqueued and its completion event recorded.
  void recorded(int slot) { used_[slot] = true; }

 private:
  unsigned next_ = 0;
  bool used_[N] = {};
};

}  // namespace prism

// Scheduling decisions of the serving loop, free of any device work: the
// first-fit arena that admits requests under the memory cap, the step budget
// of a kernel class in one time slice, and the output frames a slice produces
// and hands to the host.  Compiled into the server and into a CPU program
// (tests/serve_sched_check.cpp) that drives the same decisions with a fake
// integrator.
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <map>

namespace irk {

// First-fit allocator over [0, size) (units: doubles, in 256-byte granules)
// with coalescing of neighbouring free ranges.
class Arena {
 public:
  static constexpr int64_t kGranule = 32;  // doubles
  explicit Arena(int64_t size) {
    if (size > 0) free_[0] = size;
  }
  // Offset of n doubles, or -1 if no free range is large enough.
  int64_t alloc(int64_t n) {
    n = (n + kGranule - 1) / kGranule * kGranule;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const int64_t off = it->first, len = it->second;
        free_.erase(it);
        if (len > n) free_[off + n] = len - n;
        used_[off] = n;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    int64_t len = u->second;
    used_.erase(u);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }
  // Doubles handed out (rounded to granules).
  int64_t used() const {
    int64_t s = 0;
    for (const auto& kv : used_) s += kv.second;
    return s;
  }

 private:
  std::map<int64_t, int64_t> free_, used_;
};

// Steps per request of one kernel class in a slice: the steps expected to fit
// slice_ms at us_per_step, at least 1 and at most slice_steps.
inline int64_t slice_budget(double us_per_step, double slice_ms, int64_t slice_steps) {
  const double fit = slice_ms * 1e3 / std::max(us_per_step, 1e-3);
  const int64_t f = fit >= (double)slice_steps ? slice_steps : (int64_t)fit;
  return std::max<int64_t>(1, std::min<int64_t>(slice_steps, f));
}

// Output frames a slice stages for a request that has done `steps_done` steps
// and may advance by `budget`: frames f0 .. f1 (frame f = state after f *
// stride steps); the kernels write those the request reaches.
struct FrameWindow {
  int64_t f0, f1;
};
inline FrameWindow slice_frames(int64_t steps_done, int64_t budget, int64_t nsteps,
                                int64_t stride) {
  const int64_t end = std::min(nsteps, steps_done + budget);
  return FrameWindow{steps_done / stride, end / stride};
}

// Frames the host takes from a slice in which a request went from `old_steps`
// to `new_steps` steps: [first, last]; a request's first slice also hands
// over frame 0 (written by the setup kernel).  Empty when first > last.
inline FrameWindow harvested_frames(bool first_slice, int64_t old_steps, int64_t new_steps,
                                    int64_t stride) {
  return FrameWindow{first_slice ? 0 : old_steps / stride + 1, new_steps / stride};
}

}  // namespace irk

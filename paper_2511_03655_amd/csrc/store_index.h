// Where the batched kernels store: the step range of one launch of an
// instance and the global indices of its output frames, per-step iteration
// counts and resumable state.  Plain integer arithmetic, compiled both into
// the kernels and into a host-side check that walks the launches of a call
// (chunked, single-step, non-finite stops, evictions) and verifies that every
// index stays inside the instance's own allocation.
//
// Allocation of instance i (offsets set by the host runtime per call):
//   frames  out_off .. out_off + (nsteps / stride + 1) * dq - 1
//           (frame f holds the state after f * stride steps, [frame][dq]);
//   counts  iters_off .. iters_off + nsteps - 1 (one byte per step; only when
//           recorded, iters_off >= 0);
//   state   state_off .. state_off + (4 + S) * dq - 1
//           ([q.hi | q.lo | v.hi | v.lo] then R_prev as [component][stage]).
#pragma once

#ifndef __HIPCC_RTC__  // run-time compilation: the integer types come from device_common.h
#include <stdint.h>
#endif

#if defined(__HIPCC__)
#define IRK_HD __host__ __device__
#else
#define IRK_HD
#endif

namespace irk {

// Last step (exclusive) an instance reaches in one launch: its step count,
// capped by the launch's step budget (steps per instance per launch, <= 0:
// none) and step limit (a chunk boundary, <= 0: none); an instance that has
// stopped (status_ok false) or is already past the limit does no step.
IRK_HD inline int64_t launch_target_of(int64_t steps_done, int64_t nsteps, bool status_ok,
                                       int64_t step_budget, int64_t step_limit) {
  int64_t t = nsteps;
  if (step_budget > 0 && steps_done + step_budget < t) t = steps_done + step_budget;
  if (step_limit > 0 && step_limit < t) t = step_limit;
  if (!status_ok || t < steps_done) t = steps_done;
  return t;
}

// Component c of output frame f.
IRK_HD inline int64_t frame_index(int64_t out_off, int64_t f, int dq, int c) {
  return out_off + f * dq + c;
}

// Frames an instance that stops at a non-finite value in step step0 + 1 fills
// with NaN in this launch: first_nan_frame .. target / stride (frames of later
// launches are filled at the end of the call).
IRK_HD inline int64_t first_nan_frame(int64_t step0, int64_t stride) { return step0 / stride + 1; }
IRK_HD inline int64_t last_frame_of_launch(int64_t target, int64_t stride) {
  return target / stride;
}

// Frames by counting steps instead of dividing at every step: `next` is the
// number of the next frame and `at` the step count after which it is written
// (frame f holds the state after f * stride steps).  Set once per launch from
// the steps already done; frame_due advances it after each step and agrees
// with step % stride == 0 and f = step / stride.
struct FrameClock {
  int64_t next, at;
};
IRK_HD inline FrameClock frame_clock(int64_t steps_done, int64_t stride) {
  const int64_t f = steps_done / stride + 1;
  return FrameClock{f, f * stride};
}
IRK_HD inline bool frame_due(FrameClock& c, int64_t step, int64_t stride, int64_t& f) {
  if (step != c.at) return false;
  f = c.next;
  ++c.next;
  c.at += stride;
  return true;
}

// Iteration count of step step0 + 1.
IRK_HD inline int64_t iters_index(int64_t iters_off, int64_t step0) { return iters_off + step0; }

// Part p (0 q.hi, 1 q.lo, 2 v.hi, 3 v.lo) of component c of the resumable state.
IRK_HD inline int64_t state_index(int64_t state_off, int dq, int part, int c) {
  return state_off + (int64_t)part * dq + c;
}

// Previous-step increment of component c at stage s (S stages).
IRK_HD inline int64_t rprev_index(int64_t state_off, int dq, int c, int s, int S) {
  return state_off + 4 * (int64_t)dq + (int64_t)c * S + s;
}

}  // namespace irk

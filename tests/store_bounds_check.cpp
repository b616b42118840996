// Host-side check of the batched kernels' global stores (built with g++ by
// tests/test_store_bounds_cpu.py; no GPU).
//
// Walks the launches of integration calls the way the host runtime issues
// them -- one launch per call, chunked calls (step limits at chunk
// boundaries), the plain form (one step per launch) -- and, inside each launch,
// the step loop of an instance as the slot kernel runs it: a step that ends
// non-finite (a diverging fixed-point iteration, h * omega >> 1) writes NaN
// frames up to the launch's target and stops the instance; an evicted
// instance stops at the end of its step with its state saved; the end of a
// chunked call fills the NaN frames of later launches.  Every index comes from
// the kernels' own helpers (store_index.h) and must lie inside the instance's
// allocation; every output frame must be written at least once.  The frame
// clock that the Kepler latency kernel counts steps with (instead of dividing)
// must name the same frames as step % stride == 0 in every launch.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_2511_03655_amd/csrc/store_index.h"

namespace {

constexpr int kS = 8;

struct Inst {
  int dq;
  int64_t nsteps, stride;
  int64_t nonfinite_at;  // step (1-based) whose iteration ends non-finite, 0: never
  int64_t evict_every;   // evict at the end of every such step (0: never)
  // layout
  int64_t out_off, iters_off, state_off;
  // progress
  int64_t steps_done;
  bool ok;
};

struct Checker {
  int64_t out_total = 0, iters_total = 0, state_total = 0;
  std::vector<int> frame_written;  // per output element
  int64_t violations = 0, stores = 0;
  const char* where = "";

  void out(const Inst& in, int64_t idx) {
    ++stores;
    const int64_t lo = in.out_off, hi = in.out_off + (in.nsteps / in.stride + 1) * in.dq;
    if (idx < lo || idx >= hi) {
      if (violations++ < 5)
        std::printf("%s: frame store %lld outside [%lld, %lld)\n", where, (long long)idx,
                    (long long)lo, (long long)hi);
      return;
    }
    frame_written[idx] = 1;
  }
  void iters(const Inst& in, int64_t idx) {
    ++stores;
    if (in.iters_off < 0) return;
    if (idx < in.iters_off || idx >= in.iters_off + in.nsteps)
      if (violations++ < 5)
        std::printf("%s: count store %lld outside the instance's %lld steps\n", where,
                    (long long)idx, (long long)in.nsteps);
  }
  void state(const Inst& in, int64_t idx) {
    ++stores;
    if (idx < in.state_off || idx >= in.state_off + (4 + kS) * (int64_t)in.dq)
      if (violations++ < 5)
        std::printf("%s: state store %lld outside the instance's record\n", where,
                    (long long)idx);
  }
};

// One launch over every instance: step_budget / step_limit as the runtime
// sets them for this launch.
void launch(std::vector<Inst>& v, Checker& ck, int64_t step_budget, int64_t step_limit,
            bool evictions) {
  for (Inst& in : v) {
    const int64_t target =
        irk::launch_target_of(in.steps_done, in.nsteps, in.ok, step_budget, step_limit);
    int64_t step0 = in.steps_done;
    irk::FrameClock clk = irk::frame_clock(step0, in.stride);  // the counting form
    while (step0 < target) {
      if (in.nonfinite_at == step0 + 1) {  // non-finite increment norm in this step
        const int64_t nf = irk::last_frame_of_launch(target, in.stride);
        for (int64_t f = irk::first_nan_frame(step0, in.stride); f <= nf; ++f)
          for (int c = 0; c < in.dq; ++c) ck.out(in, irk::frame_index(in.out_off, f, in.dq, c));
        ck.iters(in, irk::iters_index(in.iters_off, step0));
        in.steps_done = step0;
        in.ok = false;
        break;
      }
      const int64_t step = step0 + 1;
      ck.iters(in, irk::iters_index(in.iters_off, step0));
      if (step % in.stride == 0)
        for (int c = 0; c < in.dq; ++c)
          ck.out(in, irk::frame_index(in.out_off, step / in.stride, in.dq, c));
      int64_t fc = -1;
      const bool due = irk::frame_due(clk, step, in.stride, fc);
      if (due != (step % in.stride == 0) || (due && fc != step / in.stride))
        if (ck.violations++ < 5)
          std::printf("%s: counted frame %lld at step %lld disagrees with step / stride\n",
                      ck.where, (long long)fc, (long long)step);
      const bool last = step >= target;
      const bool evict = !last && evictions && in.evict_every > 0 && step % in.evict_every == 0;
      if (last || evict) {
        for (int c = 0; c < in.dq; ++c) {
          for (int part = 0; part < 4; ++part)
            ck.state(in, irk::state_index(in.state_off, in.dq, part, c));
          for (int s = 0; s < kS; ++s) ck.state(in, irk::rprev_index(in.state_off, in.dq, c, s, kS));
        }
        in.steps_done = step;
        break;
      }
      step0 = step;
    }
  }
}

// End of a chunked call: NaN frames after the launch in which an instance stopped.
void nan_fill(std::vector<Inst>& v, Checker& ck) {
  for (Inst& in : v) {
    if (in.ok) continue;
    const int64_t f0 = irk::first_nan_frame(in.steps_done, in.stride);
    const int64_t f1 = irk::last_frame_of_launch(in.nsteps, in.stride);
    for (int64_t e = 0; e < (f1 - f0 + 1) * in.dq; ++e)
      ck.out(in, irk::frame_index(in.out_off, f0, in.dq, 0) + e);
  }
}

enum Mode { kOneLaunch, kChunked, kPlain };

// One call; returns the number of violations.
int64_t call(std::vector<Inst> v, Mode mode, int chunks, bool record, const char* where) {
  Checker ck;
  ck.where = where;
  int64_t max_steps = 0;
  for (Inst& in : v) {  // offsets as the runtime assigns them (instances in order)
    in.out_off = ck.out_total;
    ck.out_total += (int64_t)in.dq * (in.nsteps / in.stride + 1);
    in.iters_off = record ? ck.iters_total : -1;
    ck.iters_total += in.nsteps;
    in.state_off = ck.state_total;
    ck.state_total += (int64_t)(4 + kS) * in.dq;
    in.steps_done = 0;
    in.ok = true;
    if (in.nsteps > max_steps) max_steps = in.nsteps;
  }
  ck.frame_written.assign((size_t)ck.out_total, 0);
  for (Inst& in : v)  // frame 0: the setup kernel
    for (int c = 0; c < in.dq; ++c) ck.out(in, irk::frame_index(in.out_off, 0, in.dq, c));
  if (mode == kOneLaunch) {
    launch(v, ck, 0, 0, false);
  } else if (mode == kPlain) {
    for (int64_t s = 0; s < max_steps; ++s) launch(v, ck, 1, 0, false);
    nan_fill(v, ck);
  } else {
    const int64_t budget = (max_steps + chunks - 1) / chunks;
    for (int ch = 0; ch < chunks; ++ch) {
      const int64_t limit = (ch + 1 < chunks) ? (ch + 1) * budget : 0;
      launch(v, ck, 0, limit, ch + 1 < chunks);
    }
    nan_fill(v, ck);
  }
  for (const Inst& in : v)
    if (in.ok && in.steps_done != in.nsteps) {
      std::printf("%s: an instance ended at step %lld of %lld\n", where,
                  (long long)in.steps_done, (long long)in.nsteps);
      ++ck.violations;
    }
  int64_t unwritten = 0;
  for (int w : ck.frame_written) unwritten += (w == 0);
  if (unwritten) {
    std::printf("%s: %lld output values never written\n", where, (long long)unwritten);
    ck.violations += unwritten;
  }
  return ck.violations;
}

}  // namespace

int main() {
  const int dqs[] = {2, 9, 12, 18, 64, 192};
  const int64_t steps[] = {0, 1, 7, 64, 300, 1000, 1003};
  int64_t bad = 0, calls = 0;
  char where[160];
  for (int dq : dqs)
    for (int64_t n : steps)
      for (int64_t stride : {int64_t(1), int64_t(3), int64_t(100), n > 0 ? n : int64_t(1)}) {
        if (n % stride) continue;
        // non-finite at the first step, in the middle, at a chunk boundary,
        // at the last step, or never; evictions every 5 steps or never
        for (int64_t nfa : {int64_t(0), int64_t(1), n / 2 + 1, n / 8, n}) {
          if (nfa < 0 || nfa > n) continue;
          for (int64_t ev : {int64_t(0), int64_t(5)}) {
            // a batch: the instance under test between two ordinary ones of
            // other sizes, so that offsets are not zero
            std::vector<Inst> v = {{3, 2 * n + 3, 1, 0, 0},
                                   {dq, n, stride, nfa, ev},
                                   {5, n, n > 0 ? n : 1, 0, 7}};
            v[0].nsteps = 2 * n + 2;
            for (int mode = 0; mode < 3; ++mode)
              for (int chunks : {1, 3, 8})
                for (bool record : {false, true}) {
                  if (mode != kChunked && chunks != 1) continue;
                  std::snprintf(where, sizeof where,
                                "dq %d steps %lld stride %lld nonfinite %lld evict %lld mode %d "
                                "chunks %d record %d",
                                dq, (long long)n, (long long)stride, (long long)nfa,
                                (long long)ev, mode, chunks, (int)record);
                  bad += call(v, (Mode)mode, chunks, record, where);
                  ++calls;
                }
          }
        }
      }
  std::printf("%lld calls checked, %lld violations\n", (long long)calls, (long long)bad);
  return bad == 0 ? 0 : 1;
}

// CPU check of the serving loop's scheduling decisions (built with g++ by
// tests/test_serve_sched_cpu.py; no GPU).  The server's own helpers
// (paper_2511_03655_amd/csrc/serve_sched.h) drive a simulated server whose
// "kernel" is a fake integrator: a deterministic integer recurrence per step,
// so a request's frames are known exactly.  Checked over random streams:
//  * the arena never hands out overlapping ranges or ranges beyond the cap,
//    and first-fit fails only when no free run is long enough (against a
//    bitmap of the arena);
//  * admission is first come, first served under the cap and the slot limit;
//  * every output frame is staged and handed to the host exactly once, and a
//    request integrated over many slices (budgets from slice_budget) ends
//    with the frames of the same recurrence run in one go -- the resume is
//    exact;
//  * a request cancelled between slices keeps exactly the frames of the steps
//    it completed.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <random>
#include <vector>

#include "../paper_2511_03655_amd/csrc/serve_sched.h"

namespace {

int64_t g_fail = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      if (g_fail++ < 10) std::printf(__VA_ARGS__); \
    }                                           \
  } while (0)

uint64_t step_fn(uint64_t x, int64_t step) {  // the fake integrator's step
  return x * 6364136223846793005ull + 1442695040888963407ull + (uint64_t)step;
}

struct Req {
  int id;
  double arrival_ms;
  int64_t nsteps, stride, len;
  int cls;
  uint64_t x0;
  // server-side state
  int64_t off = -1, steps_done = 0;
  uint64_t x = 0;  // resumable state (on the device in the server)
  bool fresh = false, done = false, cancel = false;
  std::vector<uint64_t> frames;
  std::vector<int> written;  // times each frame reached the host
};

void arena_random_check(std::mt19937_64& g) {
  const int64_t size = 4096;
  irk::Arena A(size);
  std::vector<int> owner(size, -1);
  std::vector<std::pair<int64_t, int64_t>> live;  // off, len
  for (int it = 0; it < 20000; ++it) {
    if (live.empty() || g() % 3 != 0) {
      const int64_t n = 1 + (int64_t)(g() % 300);
      const int64_t off = A.alloc(n);
      const int64_t len = (n + irk::Arena::kGranule - 1) / irk::Arena::kGranule *
                          irk::Arena::kGranule;
      if (off < 0) {  // first fit failed: no free run of len granules may exist
        int64_t run = 0, best = 0;
        for (int64_t i = 0; i < size; ++i) {
          run = owner[i] < 0 ? run + 1 : 0;
          best = run > best ? run : best;
        }
        CHECK(best < len, "arena refused %lld doubles with a free run of %lld\n",
              (long long)len, (long long)best);
        continue;
      }
      CHECK(off >= 0 && off + len <= size, "arena range [%lld, %lld) outside the cap\n",
            (long long)off, (long long)(off + len));
      for (int64_t i = off; i < off + len && i < size; ++i) {
        CHECK(owner[i] < 0, "arena overlap at %lld\n", (long long)i);
        owner[i] = it;
      }
      live.push_back({off, len});
    } else {
      const size_t k = g() % live.size();
      A.release(live[k].first);
      for (int64_t i = live[k].first; i < live[k].first + live[k].second; ++i) owner[i] = -1;
      live.erase(live.begin() + k);
    }
    int64_t used = 0;
    for (auto& l : live) used += l.second;
    CHECK(used == A.used(), "arena bookkeeping %lld != %lld\n", (long long)used,
          (long long)A.used());
  }
}

void stream_check(std::mt19937_64& g, int n_req, int64_t cap, int max_resident,
                  int64_t slice_steps, double slice_ms, double cancel_p) {
  const double us_per_step[4] = {3.0, 40.0, 250.0, 1200.0};  // per class (fake timings)
  std::vector<Req> reqs(n_req);
  double t = 0;
  for (int i = 0; i < n_req; ++i) {
    Req& r = reqs[i];
    r.id = i;
    t += (double)(g() % 4000) / 1000.0;
    r.arrival_ms = t;
    r.stride = 1 + (int64_t)(g() % 50);
    r.nsteps = r.stride * (int64_t)(g() % 60);
    r.len = 8 + (int64_t)(g() % 700);
    r.cls = (int)(g() % 4);
    r.x0 = g();
    r.frames.assign(r.nsteps / r.stride + 1, 0);
    r.written.assign(r.nsteps / r.stride + 1, 0);
  }
  irk::Arena A(cap);
  std::deque<int> pending;
  std::vector<int> resident;
  int next = 0, admitted_upto = -1, finished = 0;
  double now = 0;
  int64_t slices = 0;
  while (finished < n_req) {
    if (++slices > 2000000) {  // every request finishes well before this
      CHECK(false, "stream did not drain (%d of %d finished)\n", finished, n_req);
      return;
    }
    while (next < n_req && reqs[next].arrival_ms <= now) pending.push_back(next++);
    // admission: first come, first served while memory and slots allow
    while (!pending.empty() && (int)resident.size() < max_resident) {
      Req& r = reqs[pending.front()];
      const int64_t off = A.alloc(r.len);
      if (off < 0) break;
      CHECK(r.id > admitted_upto, "request %d admitted after %d\n", r.id, admitted_upto);
      admitted_upto = r.id;
      pending.pop_front();
      r.off = off;
      r.fresh = true;
      r.x = r.x0;
      resident.push_back(r.id);
    }
    if (resident.empty()) {  // idle until the next arrival
      if (next < n_req) now = reqs[next].arrival_ms;
      continue;
    }
    for (int i : resident)  // no two resident requests share arena memory
      for (int j : resident)
        if (i < j) {
          const Req &a = reqs[i], &b = reqs[j];
          CHECK(a.off + a.len <= b.off || b.off + b.len <= a.off, "arena overlap %d %d\n", i, j);
        }
    // one slice: budgets per class, staged frame windows, fake kernels, harvest
    double slice_time = 0;
    for (int id : resident) {
      Req& r = reqs[id];
      const int64_t budget = irk::slice_budget(us_per_step[r.cls], slice_ms, slice_steps);
      CHECK(budget >= 1 && budget <= slice_steps, "budget %lld\n", (long long)budget);
      const irk::FrameWindow w = irk::slice_frames(r.steps_done, budget, r.nsteps, r.stride);
      std::vector<uint64_t> stage((size_t)(w.f1 - w.f0 + 1), 0);
      std::vector<int> staged((size_t)(w.f1 - w.f0 + 1), 0);
      if (r.fresh) {  // the setup kernel writes frame 0
        CHECK(w.f0 == 0, "fresh request's window starts at %lld\n", (long long)w.f0);
        stage[0] = r.x;
        staged[0] = 1;
      }
      const int64_t target = std::min(r.nsteps, r.steps_done + budget);
      const int64_t old = r.steps_done;
      for (int64_t s = r.steps_done; s < target; ++s) {  // the fake kernel
        r.x = step_fn(r.x, s);
        if ((s + 1) % r.stride == 0) {
          const int64_t f = (s + 1) / r.stride;
          CHECK(f >= w.f0 && f <= w.f1, "frame %lld outside the staged window\n", (long long)f);
          if (f >= w.f0 && f <= w.f1) {
            stage[f - w.f0] = r.x;
            staged[f - w.f0] = 1;
          }
        }
      }
      r.steps_done = target;
      slice_time = std::max(slice_time, us_per_step[r.cls] * (double)(target - old) / 1e3);
      const irk::FrameWindow hv = irk::harvested_frames(r.fresh, old, r.steps_done, r.stride);
      for (int64_t f = hv.f0; f <= hv.f1; ++f) {
        CHECK(f >= w.f0 && f <= w.f1 && staged[f - w.f0], "harvested frame %lld not staged\n",
              (long long)f);
        if (f >= w.f0 && f <= w.f1) r.frames[f] = stage[f - w.f0];
        r.written[f]++;
      }
      r.fresh = false;
    }
    now += slice_time + 0.05;
    // retire finished and cancelled requests
    std::vector<int> keep;
    for (int id : resident) {
      Req& r = reqs[id];
      if (r.steps_done < r.nsteps && cancel_p > 0 && (double)(g() % 1000000) / 1e6 < cancel_p)
        r.cancel = true;
      if (r.steps_done >= r.nsteps || r.cancel) {
        r.done = true;
        ++finished;
        A.release(r.off);
      } else {
        keep.push_back(id);
      }
    }
    resident.swap(keep);
  }
  // frames against the recurrence run in one go
  for (const Req& r : reqs) {
    uint64_t x = r.x0;
    const int64_t reached = r.steps_done / r.stride;
    for (int64_t f = 0; f <= r.nsteps / r.stride; ++f) {
      if (f > 0)
        for (int64_t s = (f - 1) * r.stride; s < f * r.stride; ++s) x = step_fn(x, s);
      const int want = f <= reached ? 1 : 0;  // cancelled: frames after the last step absent
      CHECK(r.written[f] == want, "request %d frame %lld written %d times (want %d)\n", r.id,
            (long long)f, r.written[f], want);
      if (f <= reached)
        CHECK(r.frames[f] == x, "request %d frame %lld differs from the one-go run\n", r.id,
              (long long)f);
    }
    CHECK(r.done, "request %d never finished\n", r.id);
  }
}

}  // namespace

int main() {
  std::mt19937_64 g(20251203);
  arena_random_check(g);
  for (int rep = 0; rep < 20; ++rep) {
    const int64_t cap = 1024 + (int64_t)(g() % 8192);
    const int max_res = 1 + (int)(g() % 40);
    const int64_t slice_steps = 1 + (int64_t)(g() % 200);
    const double slice_ms = 0.5 + (double)(g() % 400) / 10.0;
    stream_check(g, 400, cap, max_res, slice_steps, slice_ms, rep % 2 ? 0.02 : 0.0);
  }
  std::printf("%lld failures\n", (long long)g_fail);
  return g_fail == 0 ? 0 : 1;
}

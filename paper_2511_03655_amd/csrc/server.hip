// Serving loop behind irkgl16_server_* / irkgl16_submit / irkgl16_poll /
// irkgl16_wait (include/irkgl16.h): continuous batching of integration
// requests on one GPU.
//
// A serving thread repeats: admit pending requests (first come, first served)
// while their device memory fits under the cap; run one time slice, i.e. one
// batched launch per kernel class over all resident requests, the classes
// concurrently, each with a step budget sized to the target slice time from
// that class's measured time per step (newly admitted requests are first set
// up by the prepare kernel); copy the slice's statistics and output frames to
// the host; retire
// finished requests (their frames are complete on the host) and free their
// memory.  A resident request's state record never leaves the device between
// slices, and the kernels resume from it exactly, so a served request is
// bit-identical to the same request integrated alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/irkgl16.h"
#include "device_common.h"
#include "host_common.h"
#include "launch.h"
#include "serve_sched.h"

namespace {

struct Request {
  int64_t ticket = 0;
  int32_t kind = 0, n = 0, d = 0, dq = 0;
  std::vector<double> mass, coupling, q0, p0;
  double G = 1.0, eps = 0.0, beta = 0.0, h = 0.0;
  int64_t nsteps = 0, stride = 1;
  int cls = -1, S = 0;
  int64_t arena_len = 0, arena_off = -1;
  int slot = -1;
  int64_t steps_done = 0;
  std::vector<double> qf, pf;
  int32_t status = IRKGL16_OK;
  int64_t iterations = 0, nonconv = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  bool fresh = false, done = false;
  bool finish = false;  // set by the slice (worker only); published as `done` under the lock
  bool cancel = false;  // set by irkgl16_cancel (under the lock): stop after the current slice
  int64_t stage_base = 0, f0 = 0;  // this slice's frame window
  int64_t budget = 0, old_steps = 0;  // this slice's step budget, steps done before it
};

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t n, bool keep = false) {
    if (n <= bytes && p) return hipSuccess;
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 256));
    if (e != hipSuccess) return e;
    if (keep && p && bytes) (void)hipMemcpy(q, p, bytes, hipMemcpyDeviceToDevice);
    if (p) (void)hipFree(p);
    p = q;
    bytes = std::max<size_t>(n, 256);
    return hipSuccess;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct irkgl16_server {
  irkgl16_server_options opt{};
  int device = 0, num_cus = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // concurrent class launches within a slice (fork on `stream`, join back)
  static constexpr int kMaxAux = 4;
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_done;
  hipEvent_t ev_fork = nullptr;
  // per-class step time (microseconds per step of a slice), measured with
  // events around each class launch and smoothed over slices
  std::map<std::tuple<int, int, int, int>, double> step_us;
  std::vector<hipEvent_t> cls_ev;  // pairs: start, end
  irk::TuneTable tune;             // launch shapes (read at creation)
  std::chrono::steady_clock::time_point t0;

  DevBuf d_tab, d_desc, d_stat, d_arena, d_in, d_stage_q, d_stage_p, d_queue, d_heads, d_ids,
      d_large;
  int large_nmax = 0;
  std::unique_ptr<irk::Arena> arena;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::vector<Request*> resident;   // by slot
  std::vector<int> free_slots;
  std::unordered_map<int64_t, std::unique_ptr<Request>> requests;
  int64_t next_ticket = 1;
  // totals reported by irkgl16_server_stats (under the lock)
  int64_t n_slices = 0, n_finished = 0, n_cancelled = 0;
  double slice_wall_s = 0.0, slice_device_s = 0.0;
  int32_t max_resident_seen = 0;
  hipEvent_t ev_s0 = nullptr, ev_s1 = nullptr;  // device span of a slice (uploads to results)
  double last_slice_device_s = 0.0;             // worker only
  bool stopping = false;
  int device_error = 0;
  std::thread worker;

  std::vector<irk::InstDesc> h_desc;
  std::vector<irk::InstStat> h_stat;
  std::vector<double> h_stage_q, h_stage_p;

  ~irkgl16_server() {
    for (hipEvent_t e : aux_done) (void)hipEventDestroy(e);
    for (hipEvent_t e : cls_ev) (void)hipEventDestroy(e);
    for (hipStream_t sk : aux) (void)hipStreamDestroy(sk);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_s0) (void)hipEventDestroy(ev_s0);
    if (ev_s1) (void)hipEventDestroy(ev_s1);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    irk::live_streams() -= (int)aux.size() + ((own_stream && stream) ? 1 : 0);
  }
  void run();
  int slice(std::vector<Request*>& live, std::vector<Request*>& fresh);
};

static int validate(const irkgl16_problem& p) {
  int S = 0;
  if (irk::validate_problem(p) != IRKGL16_OK || irk::kernel_class(p.kind, p.n, p.d, &S) < 0)
    return IRKGL16_EINVAL;
  return IRKGL16_OK;
}

// First estimate of a class's time per step (microseconds), before any slice
// of that class has been measured.
static double model_step_us(int cls, int kind, int size) {
  switch (cls) {
    case irk::kClassSmall: return 10.0;
    case irk::kClassStage: return 8.0 + 0.6 * size;
    case irk::kClassWg:
      return kind == IRKGL16_GRAVITY ? 8.0 + (double)size * size / 150.0 : 8.0 + size / 40.0;
    default: return 200.0;
  }
}

// One time slice over the resident requests.  Called without the lock held.
// Each kernel class advances its requests by the number of steps expected to
// take opt.slice_ms (from that class's measured time per step), at least 1 and
// at most opt.slice_steps, so that fast classes are not held back by slow ones.
int irkgl16_server::slice(std::vector<Request*>& live, std::vector<Request*>& fresh) {
  const int64_t slice_steps = opt.slice_steps;
  // class of every request and the class budgets
  std::map<std::tuple<int, int, int, int>, std::vector<int32_t>> classes;
  for (Request* r : live) {
    auto key = std::make_tuple(r->cls, r->kind, r->S, r->d);
    classes[key].push_back(r->slot);
  }
  std::map<std::tuple<int, int, int, int>, int64_t> budget;
  for (auto& kv : classes) {
    const auto& key = kv.first;
    auto it = step_us.find(key);
    const double us = it != step_us.end() ? it->second
                                          : model_step_us(std::get<0>(key), std::get<1>(key),
                                                          std::get<2>(key));
    budget[key] = irk::slice_budget(us, opt.slice_ms, slice_steps);
  }
  for (Request* r : live) {
    r->budget = budget[std::make_tuple(r->cls, r->kind, r->S, r->d)];
    r->old_steps = r->steps_done;
  }
  // frame windows and staging layout
  int64_t stage_total = 0, in_total = 0;
  for (Request* r : live) {
    const irk::FrameWindow w = irk::slice_frames(r->steps_done, r->budget, r->nsteps, r->stride);
    r->f0 = w.f0;
    r->stage_base = stage_total;
    stage_total += (w.f1 - w.f0 + 1) * r->dq;
  }
  std::vector<int64_t> in_off(live.size(), 0);
  for (Request* r : fresh) in_total += r->dq;
  if (d_stage_q.ensure(sizeof(double) * std::max<int64_t>(stage_total, 1)) ||
      d_stage_p.ensure(sizeof(double) * std::max<int64_t>(stage_total, 1)) ||
      d_in.ensure(sizeof(double) * 2 * std::max<int64_t>(in_total, 1)))
    return IRKGL16_EDEVICE;
  // descriptors of every resident slot, inputs of the fresh ones
  std::vector<double> hin(2 * std::max<int64_t>(in_total, 1));
  int64_t io = 0;
  for (Request* r : fresh) {
    std::copy(r->q0.begin(), r->q0.end(), hin.begin() + io);
    std::copy(r->p0.begin(), r->p0.end(), hin.begin() + in_total + io);
    irk::InstDesc& d = h_desc[r->slot];
    d.in_off = io;
    io += r->dq;
  }
  int max_slot = 0;
  for (Request* r : live) {
    irk::InstDesc& d = h_desc[r->slot];
    d.out_off = r->stage_base - r->f0 * r->dq;
    max_slot = std::max(max_slot, r->slot + 1);
  }
  std::vector<int32_t> ids;
  for (Request* r : fresh) ids.push_back(r->slot);
  // longest remaining integration first within each class
  for (auto& kv : classes)
    std::stable_sort(kv.second.begin(), kv.second.end(), [&](int32_t x, int32_t y) {
      const Request* rx = resident[x];
      const Request* ry = resident[y];
      const double wx = (double)(rx->nsteps - rx->steps_done) * rx->n * rx->n;
      const double wy = (double)(ry->nsteps - ry->steps_done) * ry->n * ry->n;
      return wx > wy;
    });
  std::vector<int32_t> queue;
  std::vector<std::pair<std::tuple<int, int, int, int>, std::pair<int64_t, int>>> cls_list;
  for (auto& kv : classes) {
    cls_list.push_back({kv.first, {(int64_t)queue.size(), (int)kv.second.size()}});
    queue.insert(queue.end(), kv.second.begin(), kv.second.end());
  }
  if (d_queue.ensure(sizeof(int32_t) * std::max<size_t>(queue.size(), 1)) ||
      d_ids.ensure(sizeof(int32_t) * std::max<size_t>(ids.size(), 1)) ||
      d_heads.ensure(sizeof(int32_t) * std::max<size_t>(cls_list.size(), 1)))
    return IRKGL16_EDEVICE;
  hipStream_t st = stream;
#define SRV_TRY(x)                                   \
  do {                                               \
    if ((x) != hipSuccess) return IRKGL16_EDEVICE;   \
  } while (0)
  SRV_TRY(hipEventRecord(ev_s0, st));
  SRV_TRY(hipMemcpyAsync(d_desc.p, h_desc.data(), sizeof(irk::InstDesc) * max_slot,
                         hipMemcpyHostToDevice, st));
  SRV_TRY(hipMemcpyAsync(d_queue.p, queue.data(), sizeof(int32_t) * queue.size(),
                         hipMemcpyHostToDevice, st));
  SRV_TRY(hipMemsetAsync(d_heads.p, 0, sizeof(int32_t) * cls_list.size(), st));
  if (!fresh.empty()) {
    SRV_TRY(hipMemcpyAsync(d_in.p, hin.data(), sizeof(double) * 2 * in_total,
                           hipMemcpyHostToDevice, st));
    SRV_TRY(hipMemcpyAsync(d_ids.p, ids.data(), sizeof(int32_t) * ids.size(),
                           hipMemcpyHostToDevice, st));
    SRV_TRY(irk::launch_prepare(d_desc.as<irk::InstDesc>(), d_stat.as<irk::InstStat>(),
                                d_arena.as<double>(), d_arena.as<double>(), d_in.as<double>(),
                                d_in.as<double>() + in_total, d_stage_q.as<double>(),
                                d_stage_p.as<double>(), nullptr, d_heads.as<int32_t>(),
                                (int)cls_list.size(), (int)ids.size(), st,
                                d_ids.as<int32_t>()));
  }
  irk::LaunchArgs a;
  a.tab = d_tab.as<double>();
  a.desc = d_desc.as<irk::InstDesc>();
  a.stat = d_stat.as<irk::InstStat>();
  a.state = d_arena.as<double>();
  a.params = d_arena.as<double>();
  a.qout = d_stage_q.as<double>();
  a.pout = d_stage_p.as<double>();
  a.step_iters = nullptr;
  a.max_iter = opt.max_iter;
  a.exact = (opt.flags & IRKGL16_REPRODUCIBLE) ? 1 : 0;
  // batched classes concurrently on the auxiliary streams, then the
  // whole-GPU (cooperative) class alone on the slice stream
  // timing events around every class launch (pairs: start, end)
  while (cls_ev.size() < 2 * cls_list.size()) {
    hipEvent_t e;
    SRV_TRY(hipEventCreate(&e));
    cls_ev.push_back(e);
  }
  SRV_TRY(hipEventRecord(ev_fork, st));
  std::vector<char> used(aux.size(), 0);
  int aux_next = 0;
  for (size_t k = 0; k < cls_list.size(); ++k) {
    const auto& key = cls_list[k].first;
    const int cls = std::get<0>(key), kind = std::get<1>(key), sz = std::get<2>(key),
              d = std::get<3>(key);
    if (cls == irk::kClassLarge) continue;
    a.queue = d_queue.as<int32_t>() + cls_list[k].second.first;
    a.queue_len = cls_list[k].second.second;
    a.queue_head = d_heads.as<int32_t>() + k;
    a.step_budget = budget[key];
    const int j = aux_next++ % (int)aux.size();
    if (!used[j]) SRV_TRY(hipStreamWaitEvent(aux[j], ev_fork, 0));
    used[j] = 1;
    SRV_TRY(hipEventRecord(cls_ev[2 * k], aux[j]));
    irk::LaunchTune tn;
    if (cls == irk::kClassWg) tn.wg_block = tune.get(irk::wg_tune_key(kind, d, sz), 0);
    SRV_TRY(irk::launch_batched(cls, kind, sz, d, a, a.queue_len, num_cus, aux[j], tn));
    SRV_TRY(hipEventRecord(cls_ev[2 * k + 1], aux[j]));
  }
  for (size_t j = 0; j < aux.size(); ++j) {
    if (!used[j]) continue;
    SRV_TRY(hipEventRecord(aux_done[j], aux[j]));
    SRV_TRY(hipStreamWaitEvent(st, aux_done[j], 0));
  }
  for (size_t k = 0; k < cls_list.size(); ++k) {
    const int cls = std::get<0>(cls_list[k].first);
    if (cls != irk::kClassLarge) continue;
    a.queue = d_queue.as<int32_t>() + cls_list[k].second.first;
    a.queue_len = cls_list[k].second.second;
    a.queue_head = d_heads.as<int32_t>() + k;
    a.step_budget = budget[cls_list[k].first];
    SRV_TRY(hipEventRecord(cls_ev[2 * k], st));
    for (int i = 0; i < a.queue_len; ++i) {
      const int slot = queue[cls_list[k].second.first + i];
      Request* r = resident[slot];
      const int ch = irk::large_chunks(r->n, a.exact != 0, num_cus);
      SRV_TRY(irk::launch_large(a, slot, r->n, d_large.p, ch, num_cus, st,
                                tune.get(irk::large_tune_key(r->n), 0)));
    }
    SRV_TRY(hipEventRecord(cls_ev[2 * k + 1], st));
  }
  if ((int64_t)h_stage_q.size() < stage_total) {
    h_stage_q.resize(stage_total);
    h_stage_p.resize(stage_total);
  }
  SRV_TRY(hipEventRecord(ev_s1, st));
  SRV_TRY(hipMemcpyAsync(h_stat.data(), d_stat.p, sizeof(irk::InstStat) * max_slot,
                         hipMemcpyDeviceToHost, st));
  if (stage_total > 0) {
    SRV_TRY(hipMemcpyAsync(h_stage_q.data(), d_stage_q.p, sizeof(double) * stage_total,
                           hipMemcpyDeviceToHost, st));
    SRV_TRY(hipMemcpyAsync(h_stage_p.data(), d_stage_p.p, sizeof(double) * stage_total,
                           hipMemcpyDeviceToHost, st));
  }
  SRV_TRY(hipStreamSynchronize(st));
  {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev_s0, ev_s1) == hipSuccess) last_slice_device_s = 1e-3 * ms;
  }
#undef SRV_TRY
  // harvest frames and progress
  for (Request* r : live) {
    const irk::InstStat& s = h_stat[r->slot];
    const irk::FrameWindow hv = irk::harvested_frames(r->fresh, r->steps_done, s.steps_done,
                                                      r->stride);
    const int64_t fb = hv.f1;
    for (int64_t f = hv.f0; f <= fb; ++f) {
      const int64_t src = r->stage_base + (f - r->f0) * r->dq;
      std::copy(h_stage_q.begin() + src, h_stage_q.begin() + src + r->dq,
                r->qf.begin() + f * r->dq);
      std::copy(h_stage_p.begin() + src, h_stage_p.begin() + src + r->dq,
                r->pf.begin() + f * r->dq);
    }
    r->steps_done = s.steps_done;
    r->iterations = s.iterations;
    r->nonconv = s.nonconv;
    r->fresh = false;
    if (s.status != irk::kOk) {
      r->status = s.status;
      std::fill(r->qf.begin() + (fb + 1) * r->dq, r->qf.end(), std::nan(""));
      std::fill(r->pf.begin() + (fb + 1) * r->dq, r->pf.end(), std::nan(""));
      r->finish = true;
    } else if (r->steps_done >= r->nsteps) {
      r->status = r->nonconv ? IRKGL16_ENOCONV : IRKGL16_OK;
      r->finish = true;
    }
  }
  // measured time per step of each class (the longest advance in the class)
  for (size_t k = 0; k < cls_list.size(); ++k) {
    const auto& key = cls_list[k].first;
    int64_t adv = 0;
    for (int i = 0; i < cls_list[k].second.second; ++i) {
      const Request* r = resident[queue[cls_list[k].second.first + i]];
      adv = std::max<int64_t>(adv, r->steps_done - r->old_steps);
    }
    float ms = 0.f;
    if (adv > 0 && hipEventElapsedTime(&ms, cls_ev[2 * k], cls_ev[2 * k + 1]) == hipSuccess) {
      const double us = 1e3 * ms / (double)adv;
      auto it = step_us.find(key);
      step_us[key] = it == step_us.end() ? us : 0.5 * (it->second + us);
    }
  }
  return IRKGL16_OK;
}

void irkgl16_server::run() {
  (void)hipSetDevice(device);
  for (;;) {
    std::vector<Request*> live, fresh;
    {
      std::unique_lock<std::mutex> lk(mu);
      // admission: first come, first served, while memory and slots allow
      while (!pending.empty() && !free_slots.empty()) {
        Request* r = pending.front();
        const int64_t off = arena->alloc(r->arena_len);
        if (off < 0) break;
        pending.pop_front();
        r->arena_off = off;
        r->slot = free_slots.back();
        free_slots.pop_back();
        resident[r->slot] = r;
        r->t_admit = now_s(t0);
        r->fresh = true;
        // descriptor of the new request
        irk::InstDesc& d = h_desc[r->slot];
        std::memset(&d, 0, sizeof(d));
        d.kind = r->kind;
        d.n = r->n;
        d.d = r->d;
        d.G = r->G;
        d.eps = r->eps;
        d.beta = r->beta;
        d.h = r->h;
        d.nsteps = r->nsteps;
        d.stride = r->stride;
        d.iters_off = -1;
        d.state_off = off;
        int64_t po = off + (int64_t)(4 + irk::kS) * r->dq;
        d.mass_off = r->mass.empty() ? -1 : po;
        po += (int64_t)r->mass.size();
        d.coupling_off = r->coupling.empty() ? -1 : po;
        if (r->cls == irk::kClassLarge && r->n > large_nmax) {
          if (d_large.ensure(irk::large_scratch_bytes(r->n, 16)) ||
              hipMemset(d_large.p, 0, irk::large_control_bytes()) != hipSuccess) {
            device_error = IRKGL16_EDEVICE;
          }
          large_nmax = r->n;
        }
      }
      for (Request* r : resident)
        if (r) (r->fresh ? fresh : live).push_back(r);
      if (fresh.empty() && live.empty()) {
        if (stopping && pending.empty()) return;
        cv_work.wait(lk);
        continue;
      }
    }
    // parameters of fresh requests into the arena (the host copies stay alive
    // until the slice has synchronized its stream)
    std::vector<std::vector<double>> prm_host;
    for (Request* r : fresh) {
      const int64_t po = r->arena_off + (int64_t)(4 + irk::kS) * r->dq;
      std::vector<double> prm(r->mass);
      prm.insert(prm.end(), r->coupling.begin(), r->coupling.end());
      if (prm.empty()) continue;
      prm_host.push_back(std::move(prm));
      (void)hipMemcpyAsync(d_arena.as<double>() + po, prm_host.back().data(),
                           sizeof(double) * prm_host.back().size(), hipMemcpyHostToDevice, stream);
    }
    live.insert(live.end(), fresh.begin(), fresh.end());
    const auto ts = std::chrono::steady_clock::now();
    last_slice_device_s = 0.0;
    const int rc = device_error ? device_error : slice(live, fresh);
    const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
    std::lock_guard<std::mutex> lk(mu);
    ++n_slices;
    slice_wall_s += wall;
    slice_device_s += last_slice_device_s;
    max_resident_seen = std::max<int32_t>(max_resident_seen, (int32_t)live.size());
    for (Request* r : live) {
      if (rc != IRKGL16_OK && !r->finish) {
        r->status = rc;
        r->finish = true;
      }
      if (r->cancel && !r->finish) {  // frames after the last completed step stay NaN
        const int64_t fb = r->steps_done / r->stride;
        std::fill(r->qf.begin() + (fb + 1) * r->dq, r->qf.end(), std::nan(""));
        std::fill(r->pf.begin() + (fb + 1) * r->dq, r->pf.end(), std::nan(""));
        r->status = IRKGL16_ECANCELED;
        r->finish = true;
        ++n_cancelled;
      }
      if (r->finish) {
        ++n_finished;
        r->done = true;
        r->t_done = now_s(t0);
        arena->release(r->arena_off);
        resident[r->slot] = nullptr;
        free_slots.push_back(r->slot);
      }
    }
    cv_done.notify_all();
  }
}

extern "C" {

int irkgl16_server_create(irkgl16_server** out, const irkgl16_server_options* opt,
                          void* hip_stream) {
  if (!out || !opt || opt->cap_bytes <= 0) return IRKGL16_EINVAL;
  *out = nullptr;
  try {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return IRKGL16_EDEVICE;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return IRKGL16_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return IRKGL16_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return IRKGL16_EDEVICE;
    std::unique_ptr<irkgl16_server> s(new irkgl16_server());
    s->opt = *opt;
    if (s->opt.slice_steps <= 0) s->opt.slice_steps = 1000;
    if (!(s->opt.slice_ms > 0.0)) s->opt.slice_ms = 20.0;
    s->tune = irk::load_tune_table();
    if (s->opt.max_iter <= 0) s->opt.max_iter = 100;
    if (s->opt.max_resident <= 0) s->opt.max_resident = 65536;
    s->device = dev;
    s->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    s->t0 = std::chrono::steady_clock::now();
    const int64_t cap_doubles = opt->cap_bytes / (int64_t)sizeof(double);
    if (s->d_arena.ensure(sizeof(double) * (size_t)cap_doubles) != hipSuccess)
      return IRKGL16_ENOMEM;
    s->arena.reset(new irk::Arena(cap_doubles));
    const size_t R = (size_t)s->opt.max_resident;
    if (s->d_desc.ensure(sizeof(irk::InstDesc) * R) || s->d_stat.ensure(sizeof(irk::InstStat) * R) ||
        s->d_tab.ensure(sizeof(double) * irk::kTabSize))
      return IRKGL16_ENOMEM;
    std::vector<double> tab(irk::kTabSize);
    for (int i = 0; i < irk::kS; ++i) {
      tab[irk::kTabC + i] = irk::kC[i];
      tab[irk::kTabB + i] = irk::kB[i];
      for (int j = 0; j < irk::kS; ++j) {
        tab[irk::kTabEta + i * irk::kS + j] = irk::kEta[i][j];
        tab[irk::kTabMu + i * irk::kS + j] = irk::kMu[i][j];
        tab[irk::kTabNu + i * irk::kS + j] = irk::kNu[i][j];
        tab[irk::kTabK + i * irk::kS + j] = irk::kK[i][j];
      }
    }
    if (hipMemcpy(s->d_tab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
      return IRKGL16_EDEVICE;
    s->h_desc.resize(R);
    s->h_stat.resize(R);
    s->resident.assign(R, nullptr);
    for (int i = (int)R - 1; i >= 0; --i) s->free_slots.push_back(i);
    if (hip_stream) {
      s->stream = (hipStream_t)hip_stream;
    } else {
      if (hipStreamCreate(&s->stream) != hipSuccess) return IRKGL16_EDEVICE;
      s->own_stream = true;
      ++irk::live_streams();
    }
    for (int k = 0; k < irkgl16_server::kMaxAux; ++k) {
      hipStream_t sk;
      hipEvent_t ek;
      if (hipStreamCreateWithFlags(&sk, hipStreamNonBlocking) != hipSuccess) return IRKGL16_EDEVICE;
      s->aux.push_back(sk);
      ++irk::live_streams();
      if (hipEventCreateWithFlags(&ek, hipEventDisableTiming) != hipSuccess) return IRKGL16_EDEVICE;
      s->aux_done.push_back(ek);
    }
    if (hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&s->ev_s0) != hipSuccess || hipEventCreate(&s->ev_s1) != hipSuccess)
      return IRKGL16_EDEVICE;
    irkgl16_server* raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = raw;
    return IRKGL16_OK;
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

int irkgl16_submit(irkgl16_server* s, const irkgl16_problem* prob, const double* q0,
                   const double* p0, double h, int64_t nsteps, int64_t out_stride,
                   int64_t* ticket) {
  if (!s || !prob || !q0 || !p0 || !ticket) return IRKGL16_EINVAL;
  if (validate(*prob) != IRKGL16_OK) return IRKGL16_EINVAL;
  if (!std::isfinite(h) || h == 0.0 || nsteps < 0 || out_stride < 1 || nsteps % out_stride)
    return IRKGL16_EINVAL;
  try {
    std::unique_ptr<Request> r(new Request());
    r->kind = prob->kind;
    r->n = prob->n;
    r->d = prob->d;
    r->dq = prob->n * prob->d;
    r->G = prob->G;
    r->eps = prob->eps;
    r->beta = prob->beta;
    if (prob->mass && prob->kind != IRKGL16_KEPLER) r->mass.assign(prob->mass, prob->mass + prob->n);
    if (prob->coupling && prob->kind == IRKGL16_CHAIN)
      r->coupling.assign(prob->coupling, prob->coupling + prob->n + 1);
    r->q0.assign(q0, q0 + r->dq);
    r->p0.assign(p0, p0 + r->dq);
    r->h = h;
    r->nsteps = nsteps;
    r->stride = out_stride;
    r->cls = irk::kernel_class(r->kind, r->n, r->d, &r->S);
    r->arena_len = (int64_t)(4 + irk::kS) * r->dq + (int64_t)r->mass.size() +
                   (int64_t)r->coupling.size();
    if (r->arena_len * (int64_t)sizeof(double) > s->opt.cap_bytes) return IRKGL16_EINVAL;
    const int64_t nf = nsteps / out_stride + 1;
    r->qf.assign((size_t)(nf * r->dq), 0.0);
    r->pf.assign((size_t)(nf * r->dq), 0.0);
    std::lock_guard<std::mutex> lk(s->mu);
    r->ticket = s->next_ticket++;
    r->t_submit = now_s(s->t0);
    *ticket = r->ticket;
    s->pending.push_back(r.get());
    s->requests[r->ticket] = std::move(r);
    s->cv_work.notify_one();
    return IRKGL16_OK;
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  }
}

int irkgl16_poll(irkgl16_server* s, int64_t ticket, int32_t* done) {
  if (!s || !done) return IRKGL16_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return IRKGL16_EINVAL;
  *done = it->second->done ? 1 : 0;
  return IRKGL16_OK;
}

int irkgl16_wait(irkgl16_server* s, int64_t ticket, double* q_out, double* p_out,
                 irkgl16_request_info* info) {
  if (!s) return IRKGL16_EINVAL;
  std::unique_ptr<Request> r;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return IRKGL16_EINVAL;
    Request* raw = it->second.get();
    s->cv_done.wait(lk, [&] { return raw->done; });
    r = std::move(it->second);
    s->requests.erase(it);
  }
  if (q_out) std::memcpy(q_out, r->qf.data(), sizeof(double) * r->qf.size());
  if (p_out) std::memcpy(p_out, r->pf.data(), sizeof(double) * r->pf.size());
  if (info) {
    info->status = r->status;
    info->steps = r->steps_done;
    info->iterations = r->iterations;
    info->submit_s = r->t_submit;
    info->admit_s = r->t_admit;
    info->done_s = r->t_done;
  }
  return r->status;
}

int irkgl16_cancel(irkgl16_server* s, int64_t ticket) {
  if (!s) return IRKGL16_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return IRKGL16_EINVAL;
  Request* r = it->second.get();
  if (r->done) return IRKGL16_OK;
  auto pq = std::find(s->pending.begin(), s->pending.end(), r);
  if (pq != s->pending.end()) {  // never admitted: no frame beyond the initial state
    s->pending.erase(pq);
    std::fill(r->qf.begin(), r->qf.end(), std::nan(""));
    std::fill(r->pf.begin(), r->pf.end(), std::nan(""));
    std::copy(r->q0.begin(), r->q0.end(), r->qf.begin());
    std::copy(r->p0.begin(), r->p0.end(), r->pf.begin());
    r->status = IRKGL16_ECANCELED;
    r->done = true;
    r->t_done = now_s(s->t0);
    ++s->n_finished;
    ++s->n_cancelled;
    s->cv_done.notify_all();
    return IRKGL16_OK;
  }
  r->cancel = true;  // resident: stops when the current slice ends
  return IRKGL16_OK;
}

int irkgl16_server_stats(irkgl16_server* s, irkgl16_server_info* out) {
  if (!s || !out) return IRKGL16_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  out->slices = s->n_slices;
  out->slice_wall_s = s->slice_wall_s;
  out->slice_device_s = s->slice_device_s;
  out->requests_done = s->n_finished;
  out->requests_cancelled = s->n_cancelled;
  out->max_resident = s->max_resident_seen;
  int32_t res = 0;
  for (Request* r : s->resident) res += r ? 1 : 0;
  out->resident = res;
  out->pending = (int32_t)s->pending.size();
  return IRKGL16_OK;
}

void irkgl16_server_destroy(irkgl16_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  delete s;
}

}  // extern "C"

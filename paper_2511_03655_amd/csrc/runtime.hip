// Host runtime behind the C ABI declared in include/irkgl16.h.
//
// A context owns the device copies of every instance's problem constants, a
// resumable state arena (q, v as two-double values plus the previous step's
// stage increments), per-instance statistics and one work queue per kernel
// class.  irkgl16_integrate uploads per-call step sizes and counts, launches
// the setup kernel and one persistent kernel per class on the context's
// stream, and (in host-pointer mode) copies the output frames back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/irkgl16.h"
#include "device_common.h"
#include "host_common.h"
#include "launch.h"


namespace {

struct KernelClass {
  int cls = -1;   // irk::kClass*
  int kind = 0, size = 0, d = 0;  // size: see irk::kernel_class
  irk::LaunchTune tune;           // launch shape from the tuning table
  std::vector<int32_t> ids;
  int64_t queue_off = 0;
};

// Work of one step of an instance, up to a constant factor (orders a class's
// queue so that the longest integrations start first).
double step_work(const irk::InstDesc& d) {
  const double n = d.n;
  return d.kind == IRKGL16_GRAVITY ? n * n * d.d : n * d.d;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t ensure(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (n == 0) n = 8;
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

}  // namespace

namespace irk {

int validate_problem(const irkgl16_problem& p) {
  auto finite = [](double x) { return std::isfinite(x); };
  if (p.n < 1 || p.d < 1 || p.d > 3) return IRKGL16_EINVAL;
  switch (p.kind) {
    case IRKGL16_KEPLER:
      if (p.n != 1 || p.d < 2 || !finite(p.G)) return IRKGL16_EINVAL;
      return IRKGL16_OK;
    case IRKGL16_GRAVITY:
      if (!p.mass || !finite(p.G) || !finite(p.eps) || p.eps < 0.0) return IRKGL16_EINVAL;
      for (int a = 0; a < p.n; ++a)
        if (!(p.mass[a] > 0.0) || !finite(p.mass[a])) return IRKGL16_EINVAL;
      return IRKGL16_OK;
    case IRKGL16_CHAIN:
      if (p.d != 1 || !finite(p.beta)) return IRKGL16_EINVAL;
      if (p.mass)
        for (int a = 0; a < p.n; ++a)
          if (!(p.mass[a] > 0.0) || !finite(p.mass[a])) return IRKGL16_EINVAL;
      if (p.coupling)
        for (int a = 0; a <= p.n; ++a)
          if (!finite(p.coupling[a])) return IRKGL16_EINVAL;
      return IRKGL16_OK;
    default:
      return IRKGL16_EINVAL;
  }
}

std::atomic<int>& live_streams() {
  static std::atomic<int> n{0};
  return n;
}

int summarize_stats(const InstStat* h_stat, int32_t n, irkgl16_stats* stats) {
  int worst = IRKGL16_OK;
  int64_t steps = 0, iters = 0, nonconv = 0;
  int32_t maxk = 0, nnf = 0;
  for (int32_t i = 0; i < n; ++i) {
    const InstStat& s = h_stat[i];
    steps += s.steps_done;
    iters += s.iterations;
    nonconv += s.nonconv;
    maxk = std::max(maxk, s.max_k);
    int st = s.status;
    if (st == kOk && s.nonconv > 0) st = IRKGL16_ENOCONV;
    if (s.status == kNonFinite) ++nnf;
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (st > 0 && worst == IRKGL16_OK) worst = st;
    if (stats) {
      if (stats->inst_iterations) stats->inst_iterations[i] = s.iterations;
      if (stats->inst_status) stats->inst_status[i] = st;
    }
  }
  if (stats) {
    stats->steps = steps;
    stats->iterations = iters;
    stats->nonconverged_steps = nonconv;
    stats->max_k = maxk;
    stats->n_nonfinite = nnf;
  }
  return worst;
}

}  // namespace irk

struct irkgl16_ctx {
  int device = 0;
  int num_cus = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bool halves = false;  // a class was split in two (per-class chunk pipelines)
  int32_t n_inst = 0;
  int32_t max_iter = 100;
  bool record = false;
  uint32_t flags = 0;

  std::vector<irk::InstDesc> desc;
  std::vector<int32_t> dq;
  std::vector<KernelClass> classes;
  int64_t total_dq = 0;

  DevBuf d_tab, d_desc, d_stat, d_state, d_params, d_queue, d_heads, d_plainq;
  DevBuf d_queue2, d_prev;  // chunked calls: reordered queues, per-instance counters
  DevBuf d_qprom, d_counts, d_heads_prom;  // promoted queues, queue lengths, their heads
  DevBuf d_evicted;                         // per instance: evicted by the small-system kernel
  int chunks = 0;            // chunks per call (0: automatic)
  int max_chunks = 8;        // automatic chunk count at most this
  double promote_k = 5.0;    // promotion threshold, iterations per step (0: never)
  double evict_k = 12.0;     // mid-chunk eviction threshold, recent iterations per step (0: never)
  DevBuf d_q0, d_p0, d_qout, d_pout, d_iters, d_large;
  int large_nmax = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // concurrent class launches: fork event on `stream`, one stream + join event per class slot
  static constexpr int kMaxAux = 4;
  std::vector<hipStream_t> aux;
  std::vector<hipEvent_t> aux_done;
  hipEvent_t ev_fork = nullptr;

  std::vector<int32_t> h_queue;
  irk::TuneTable tune;  // launch shapes (read at creation)
  irk::UserKernel* user = nullptr;  // run-time compiled force (irkgl16_create_user)
  bool ode = false;                 // first-order form: state y only, no p in or out
  int stages = 8;                   // s of the s-stage member (2, 4, 6: user contexts only)
  int method = 0;                   // IRKGL16_STRANG / IRKGL16_SUZ90: explicit baselines

  // last call
  bool have_last = false;
  bool last_synced = false;
  int64_t last_iters_total = 0;
  std::vector<int64_t> last_nsteps;
  std::vector<irk::InstStat> h_stat;
  float last_ms = 0.f;

  ~irkgl16_ctx() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (hipEvent_t e : aux_done) (void)hipEventDestroy(e);
    for (hipStream_t sk : aux) (void)hipStreamDestroy(sk);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
    irk::live_streams() -= (int)aux.size() + ((own_stream && stream) ? 1 : 0);
    irk::user_kernel_free(user);
  }
};

#define HIP_TRY(expr)                                   \
  do {                                                  \
    hipError_t _e = (expr);                             \
    if (_e != hipSuccess) return IRKGL16_EDEVICE;       \
  } while (0)

static int alloc_try(DevBuf& b, size_t n) {
  hipError_t e = b.ensure(n);
  if (e == hipErrorOutOfMemory) return IRKGL16_ENOMEM;
  if (e != hipSuccess) return IRKGL16_EDEVICE;
  return IRKGL16_OK;
}

#define ALLOC_TRY(buf, n)                  \
  do {                                     \
    int _rc = alloc_try((buf), (n));       \
    if (_rc != IRKGL16_OK) return _rc;     \
  } while (0)

// A user force (irkgl16_create_user): every instance has Dq = dq components
// and n_params parameters.
struct UserSpec {
  const char* src;
  int32_t dq, n_params;
  const double* params;  // n_inst x n_params
  bool ode;              // first-order right-hand side f(t, y) (irkgl16_create_ode)
};

// Chunks per call for a chunked class: `fixed` if positive, else one chunk
// per 64 steps of its longest integration, at most max_chunks (8 unless the
// tuning table says otherwise: with mid-chunk eviction, more chunk boundaries
// cost more than they catch; 8 chunks ran the 65,536-system ensemble 3-4 %
// faster than 16, and 4, 6, 10, 12, 24 and 32 slower than 8).
static int chunk_count(int fixed, int64_t max_steps, int max_chunks) {
  constexpr int64_t kMinChunkSteps = 64;
  if (max_steps <= 0) return 1;
  if (fixed > 0) return (int)std::min<int64_t>(fixed, max_steps);
  return (int)std::max<int64_t>(
      1, std::min<int64_t>(std::max(1, max_chunks), max_steps / kMinChunkSteps));
}

// A gravitational few-body instance whose last chunk needed many iterations
// per step can run its next chunk on the stage-parallel kernel (a wavefront
// per system instead of 8 lanes: a much shorter iteration); the two kernels
// compute the same arithmetic, so results do not depend on which one ran a
// step.
static bool promotable(const irkgl16_ctx* c, const KernelClass& kc) {
  return c->promote_k > 0.0 && kc.cls == irk::kClassSmall && kc.kind == irk::kGravity &&
         irk::stage_class_supported(kc.kind, kc.size, kc.d);
}

static int create_impl(irkgl16_ctx** out, const irkgl16_problem* probs, int32_t n_inst,
                       const irkgl16_options* opt, void* hip_stream,
                       const UserSpec* user = nullptr) {
  if (!out) return IRKGL16_EINVAL;
  *out = nullptr;
  if (n_inst < 0 || (n_inst > 0 && !probs)) return IRKGL16_EINVAL;
  if (user) {
    if (!user->src || !irk::user_dq_supported(user->dq) || user->n_params < 0 ||
        (user->n_params > 0 && n_inst > 0 && !user->params))
      return IRKGL16_EINVAL;
    for (int64_t k = 0; k < (int64_t)n_inst * user->n_params; ++k)
      if (!std::isfinite(user->params[k])) return IRKGL16_EINVAL;
  } else {
    for (int32_t i = 0; i < n_inst; ++i) {
      int rc = irk::validate_problem(probs[i]);
      if (rc != IRKGL16_OK) return rc;
    }
  }
  {
    // The lower-order members run only on the run-time compiled kernels.
    const int st = (opt && opt->stages > 0) ? opt->stages : irk::kS;
    if ((opt && opt->stages < 0) || !irk::stages_supported(st) || (st != irk::kS && !user))
      return IRKGL16_EINVAL;
    // The explicit baselines exist for second-order user forces only.
    const int method = opt ? opt->method : 0;
    if (method < 0 || method > IRKGL16_SUZ90 ||
        (method != 0 && (!user || user->ode || (opt->stages != 0 && opt->stages != irk::kS))))
      return IRKGL16_EINVAL;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return IRKGL16_EDEVICE;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return IRKGL16_EDEVICE;

  irkgl16_ctx* c = new (std::nothrow) irkgl16_ctx();
  if (!c) return IRKGL16_ENOMEM;
  c->device = dev;
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
  c->n_inst = n_inst;
  if (opt) {
    c->max_iter = opt->max_iter > 0 ? opt->max_iter : 100;
    c->record = opt->record_iters != 0;
    c->flags = opt->flags;
    c->stages = opt->stages > 0 ? opt->stages : irk::kS;
    c->method = opt->method;
  }
  if (c->max_iter > 255 && c->record) c->max_iter = 255;  // counts stored as bytes

  auto fail = [&](int rc) {
    delete c;
    return rc;
  };


  // Problem constants and state layout.
  std::vector<double> params;
  c->desc.resize(n_inst);
  c->dq.resize(n_inst);
  int64_t state_off = 0;
  std::map<std::tuple<int, int, int, int>, int> cls_index;
  for (int32_t i = 0; i < n_inst; ++i) {
    const irkgl16_problem& p = probs[i];
    irk::InstDesc& d = c->desc[i];
    std::memset(&d, 0, sizeof(d));
    d.kind = p.kind;
    d.n = p.n;
    d.d = p.d;
    d.G = p.G;
    d.eps = p.eps;
    d.beta = p.beta;
    d.mass_off = -1;
    d.coupling_off = -1;
    if (p.mass && p.kind != IRKGL16_KEPLER) {
      d.mass_off = (int64_t)params.size();
      params.insert(params.end(), p.mass, p.mass + p.n);
    }
    if (p.coupling && p.kind == IRKGL16_CHAIN) {
      d.coupling_off = (int64_t)params.size();
      params.insert(params.end(), p.coupling, p.coupling + p.n + 1);
    }
    if (user && user->n_params > 0) {  // the force's parameters, via the coupling offset
      d.coupling_off = (int64_t)params.size();
      const double* pp = user->params + (int64_t)i * user->n_params;
      params.insert(params.end(), pp, pp + user->n_params);
    }
    const int dqi = p.n * p.d;
    c->dq[i] = dqi;
    d.in_off = c->total_dq;
    c->total_dq += dqi;
    d.state_off = state_off;
    state_off += (int64_t)(4 + irk::kS) * dqi;
    // kernel class
    int size = 0;
    const int cl = user ? irk::kClassUser : irk::kernel_class(p.kind, p.n, p.d, &size);
    if (cl < 0) return fail(IRKGL16_EINVAL);
    if (cl == irk::kClassLarge) c->large_nmax = std::max(c->large_nmax, (int)p.n);
    auto key = std::make_tuple(cl, (int)p.kind, size, (int)p.d);
    auto it = cls_index.find(key);
    int ci;
    if (it == cls_index.end()) {
      ci = (int)c->classes.size();
      cls_index[key] = ci;
      KernelClass kc;
      kc.cls = cl;
      kc.kind = p.kind;
      kc.size = size;
      kc.d = p.d;
      c->classes.push_back(kc);
    } else {
      ci = it->second;
    }
    c->classes[ci].ids.push_back(i);
  }
  if (user) {
    std::string log;
    const int rc = irk::user_kernel_create(user->src, user->dq,
                                           (c->flags & IRKGL16_REPRODUCIBLE) != 0, user->ode,
                                           c->stages, c->method, &c->user, &log);
    c->ode = user->ode;
    if (rc != 0) return fail(rc == -1 ? IRKGL16_EINVAL : IRKGL16_EDEVICE);
  }
  // Launch shapes and call schedule from the tuning table (the environment
  // variables below override the schedule keys).
  c->tune = irk::load_tune_table();
  c->max_chunks = std::max(1, c->tune.get("sched/max_chunks", 8));
  c->promote_k = std::max(0, c->tune.get("sched/promote_k10", 50)) / 10.0;
  c->evict_k = std::max(0, c->tune.get("sched/evict_k10", 120)) / 10.0;
  // Chunks per call of the batched classes (0 or unset: automatic).
  if (const char* ch = std::getenv("IRKGL16_CHUNKS")) c->chunks = std::max(0, std::atoi(ch));
  // Iterations per step from which a small-system instance moves to the
  // stage-parallel kernel for the next chunk (0: never).
  if (const char* pk = std::getenv("IRKGL16_PROMOTE_K")) c->promote_k = std::max(0.0, std::atof(pk));
  // Recent iterations per step from which the small-system kernel stops an
  // instance mid-chunk for promotion at the next chunk (0: never).
  if (const char* ek = std::getenv("IRKGL16_EVICT_K")) c->evict_k = std::max(0.0, std::atof(ek));
  // A promotable few-body class with at least twice as many instances as the
  // GPU holds slots for (8 wavefronts of 8 slots per CU) runs as two halves
  // (alternate instances), each with its own stream, chunk pipeline and
  // promotion stream: while one half drains the end of a chunk, the other's
  // wavefronts take the freed slots.  That needs the two halves' streams on
  // hardware queues of their own, so it is done only while this process's
  // streams (the caller's and the default one, the library's live ones and
  // this context's) fit in GPU_MAX_HW_QUEUES; IRKGL16_HALVES=0/1 overrides.
  bool halves = false;
  if (const char* hv = std::getenv("IRKGL16_HALVES")) {
    halves = std::atoi(hv) != 0;
  } else {
    int hwq = 4;
    if (const char* q = std::getenv("GPU_MAX_HW_QUEUES")) hwq = std::max(1, std::atoi(q));
    const int own = irkgl16_ctx::kMaxAux + (hip_stream ? 0 : 1);
    halves = irk::live_streams().load() + own + 2 <= hwq;
  }
  if (halves) {
    const size_t resident = (size_t)8 * 8 * (size_t)c->num_cus;
    const size_t n_cls = c->classes.size();
    for (size_t k = 0; k < n_cls; ++k) {
      KernelClass& kc = c->classes[k];
      if (!promotable(c, kc) || kc.ids.size() < 2 * resident) continue;
      KernelClass half = kc;
      half.ids.clear();
      std::vector<int32_t> keep;
      for (size_t t = 0; t < kc.ids.size(); ++t) (t % 2 ? half.ids : keep).push_back(kc.ids[t]);
      kc.ids.swap(keep);
      c->classes.push_back(half);
      c->halves = true;
    }
  }
  for (auto& kc : c->classes)
    if (kc.cls == irk::kClassWg)
      kc.tune.wg_block = c->tune.get(irk::wg_tune_key(kc.kind, kc.d, kc.size), 0);
  // Queue storage (filled per call, in longest-integration-first order).
  size_t queue_len = 0;
  for (auto& kc : c->classes) {
    kc.queue_off = (int64_t)queue_len;
    queue_len += kc.ids.size();
  }
  std::vector<int32_t> plainq(n_inst);
  for (int32_t i = 0; i < n_inst; ++i) plainq[i] = i;

  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreate(&c->stream) != hipSuccess) return fail(IRKGL16_EDEVICE);
    c->own_stream = true;
    ++irk::live_streams();
  }
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess)
    return fail(IRKGL16_EDEVICE);

  int rc;
  if (c->large_nmax > 0) {
    if ((rc = alloc_try(c->d_large, irk::large_scratch_bytes(c->large_nmax, 16)))) return fail(rc);
    if (hipMemset(c->d_large.p, 0, irk::large_control_bytes()) != hipSuccess)
      return fail(IRKGL16_EDEVICE);
  }
  if ((rc = alloc_try(c->d_desc, sizeof(irk::InstDesc) * (size_t)std::max(n_inst, 1))) ||
      (rc = alloc_try(c->d_stat, sizeof(irk::InstStat) * (size_t)std::max(n_inst, 1))) ||
      (rc = alloc_try(c->d_state, sizeof(double) * (size_t)std::max<int64_t>(state_off, 1))) ||
      (rc = alloc_try(c->d_params, sizeof(double) * std::max<size_t>(params.size(), 1))) ||
      (rc = alloc_try(c->d_queue, sizeof(int32_t) * std::max<size_t>(queue_len, 1))) ||
      (rc = alloc_try(c->d_queue2, sizeof(int32_t) * std::max<size_t>(queue_len, 1))) ||
      (rc = alloc_try(c->d_prev, sizeof(int64_t) * 2 * (size_t)std::max(n_inst, 1))) ||
      (rc = alloc_try(c->d_qprom, sizeof(int32_t) * std::max<size_t>(queue_len, 1))) ||
      (rc = alloc_try(c->d_counts, sizeof(int32_t) * 2 * std::max<size_t>(c->classes.size(), 1))) ||
      (rc = alloc_try(c->d_heads_prom, sizeof(int32_t) * std::max<size_t>(c->classes.size(), 1))) ||
      (rc = alloc_try(c->d_evicted, (size_t)std::max(n_inst, 1))) ||
      (rc = alloc_try(c->d_plainq, sizeof(int32_t) * std::max<size_t>(plainq.size(), 1))) ||
      (rc = alloc_try(c->d_heads, sizeof(int32_t) * std::max<size_t>(c->classes.size(), 1))))
    return fail(rc);
  {
    // Coefficient table of the context's member (layout Tab<s> of device_common.h).
    const double* src = irk::kTabS8;
    size_t n = sizeof(irk::kTabS8) / sizeof(double);
    if (c->stages == 2) src = irk::kTabS2, n = sizeof(irk::kTabS2) / sizeof(double);
    if (c->stages == 4) src = irk::kTabS4, n = sizeof(irk::kTabS4) / sizeof(double);
    if (c->stages == 6) src = irk::kTabS6, n = sizeof(irk::kTabS6) / sizeof(double);
    if (c->method == IRKGL16_STRANG)
      src = irk::kSplitStrang, n = sizeof(irk::kSplitStrang) / sizeof(double);
    if (c->method == IRKGL16_SUZ90)
      src = irk::kSplitSuz90, n = sizeof(irk::kSplitSuz90) / sizeof(double);
    std::vector<double> tab(irk::kTabSize, 0.0);
    std::copy(src, src + n, tab.begin());
    if ((rc = alloc_try(c->d_tab, sizeof(double) * tab.size()))) return fail(rc);
    if (hipMemcpy(c->d_tab.p, tab.data(), sizeof(double) * tab.size(), hipMemcpyHostToDevice) !=
        hipSuccess)
      return fail(IRKGL16_EDEVICE);
  }
  if (!params.empty() &&
      hipMemcpy(c->d_params.p, params.data(), sizeof(double) * params.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return fail(IRKGL16_EDEVICE);
  if (!plainq.empty() &&
      hipMemcpy(c->d_plainq.p, plainq.data(), sizeof(int32_t) * plainq.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return fail(IRKGL16_EDEVICE);
  // Auxiliary streams: the classes' persistent kernels run concurrently.
  const int n_aux = irkgl16_ctx::kMaxAux;
  for (int k = 0; k < n_aux; ++k) {
    hipStream_t sk;
    hipEvent_t ek;
    if (hipStreamCreateWithFlags(&sk, hipStreamNonBlocking) != hipSuccess) return fail(IRKGL16_EDEVICE);
    c->aux.push_back(sk);
    ++irk::live_streams();
    if (hipEventCreateWithFlags(&ek, hipEventDisableTiming) != hipSuccess) return fail(IRKGL16_EDEVICE);
    c->aux_done.push_back(ek);
  }
  if (hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess)
    return fail(IRKGL16_EDEVICE);
  *out = c;
  return IRKGL16_OK;
}

// Estimated duration of a batched class in a call, in arbitrary units: its
// longest integration, steps times the latency of one step of one instance
// on that class's kernel (few-body: about constant; stage-parallel: the
// source loop over the padded body count; workgroup kernel: the source loop
// over the bodies, or the chain's neighbour terms).  Orders the classes over
// the auxiliary streams when they outnumber them.
static double class_estimate(const KernelClass& kc, const int64_t* nsteps) {
  double lat = 1.0;
  if (kc.cls == irk::kClassStage) lat = kc.size / 8.0;
  if (kc.cls == irk::kClassWg) lat = kc.kind == irk::kGravity ? kc.size / 16.0 : 1.0;
  int64_t m = 0;
  for (int32_t id : kc.ids) m = std::max(m, nsteps[id]);
  return lat * (double)m;
}

static irk::LaunchArgs base_args(irkgl16_ctx* c, double* qout, double* pout) {
  irk::LaunchArgs a;
  a.tab = c->d_tab.as<double>();
  a.desc = c->d_desc.as<irk::InstDesc>();
  a.stat = c->d_stat.as<irk::InstStat>();
  a.state = c->d_state.as<double>();
  a.params = c->d_params.as<double>();
  a.qout = qout;
  a.pout = pout;
  a.step_iters = c->record ? c->d_iters.as<uint8_t>() : nullptr;
  a.queue = nullptr;
  a.queue_len = 0;
  a.max_iter = c->max_iter;
  a.queue_head = nullptr;
  a.step_budget = 0;
  a.exact = (c->flags & IRKGL16_REPRODUCIBLE) ? 1 : 0;
  return a;
}

static hipError_t launch_class(irkgl16_ctx* c, const KernelClass& kc, const irk::LaunchArgs& a,
                               int n_items, hipStream_t st) {
  if (kc.cls == irk::kClassLarge) {
    // One cooperative whole-GPU launch per instance, in queue order.
    std::vector<int32_t> ids;
    if (a.queue_head)
      ids.assign(kc.ids.begin(), kc.ids.end());
    else  // plain form: the single instance is identified by its queue position
      ids.push_back((int32_t)(a.queue - c->d_plainq.as<int32_t>()));
    for (int32_t id : ids) {
      const int n = c->desc[id].n;
      const int ch = irk::large_chunks(n, a.exact != 0, c->num_cus);
      hipError_t e = irk::launch_large(a, id, n, c->d_large.p, ch, c->num_cus, st,
                                       c->tune.get(irk::large_tune_key(n), 0));
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (kc.cls == irk::kClassUser) return irk::launch_user(*c->user, a, n_items, c->num_cus, st);
  return irk::launch_batched(kc.cls, kc.kind, kc.size, kc.d, a, n_items, c->num_cus, st, kc.tune);
}

// Plain form, graph replay: capture one single-step launch per instance (all
// batched classes, as parallel branches), then replay the graph once per step;
// the kernels read each instance's progress from device memory and do nothing
// for an instance that has reached its step count.  Cooperative (whole-GPU)
// launches are issued directly after each replay.
static hipError_t plain_graph_steps(irkgl16_ctx* c, const irk::LaunchArgs& a,
                                    const int64_t* nsteps) {
  int64_t smax = 0;
  bool any_batched = false, any_large = false;
  for (const auto& kc : c->classes)
    for (int32_t id : kc.ids) {
      smax = std::max(smax, nsteps[id]);
      (kc.cls == irk::kClassLarge ? any_large : any_batched) = true;
    }
  if (smax == 0) return hipSuccess;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipSuccess;
  if (any_batched) {
    // The step's launches are independent of each other: they are captured as
    // parallel branches (round robin over the auxiliary streams, forked from
    // and joined back into the context stream).
    e = hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return e;
    const int nb = std::max<int>(1, (int)c->aux.size());
    std::vector<char> used(c->aux.size(), 0);
    if (!c->aux.empty()) e = hipEventRecord(c->ev_fork, c->stream);
    int next = 0;
    for (const auto& kc : c->classes) {
      if (kc.cls == irk::kClassLarge) continue;
      for (int32_t id : kc.ids) {
        irk::LaunchArgs pa = a;
        pa.queue = c->d_plainq.as<int32_t>() + id;
        pa.queue_len = 1;
        pa.queue_head = nullptr;
        pa.step_budget = 1;
        hipStream_t sj = c->stream;
        if (!c->aux.empty()) {
          const int j = next++ % nb;
          sj = c->aux[j];
          if (e == hipSuccess && !used[j]) e = hipStreamWaitEvent(sj, c->ev_fork, 0);
          used[j] = 1;
        }
        if (e == hipSuccess) e = launch_class(c, kc, pa, 1, sj);
      }
    }
    for (size_t j = 0; j < c->aux.size(); ++j) {
      if (!used[j] || e != hipSuccess) continue;
      e = hipEventRecord(c->aux_done[j], c->aux[j]);
      if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->aux_done[j], 0);
    }
    const hipError_t ec = hipStreamEndCapture(c->stream, &graph);
    if (e == hipSuccess) e = ec;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  }
  for (int64_t s = 0; s < smax && e == hipSuccess; ++s) {
    if (exec) e = hipGraphLaunch(exec, c->stream);
    if (!any_large) continue;
    for (const auto& kc : c->classes) {
      if (kc.cls != irk::kClassLarge) continue;
      for (int32_t id : kc.ids) {
        if (s >= nsteps[id] || e != hipSuccess) continue;
        irk::LaunchArgs pa = a;
        pa.queue = c->d_plainq.as<int32_t>() + id;
        pa.queue_len = 1;
        pa.queue_head = nullptr;
        pa.step_budget = 1;
        e = launch_class(c, kc, pa, 1, c->stream);
      }
    }
  }
  if (exec) {
    const hipError_t es = hipStreamSynchronize(c->stream);  // graph done before destroy
    if (e == hipSuccess) e = es;
    (void)hipGraphExecDestroy(exec);
  }
  if (graph) (void)hipGraphDestroy(graph);
  return e;
}

static int integrate_impl(irkgl16_ctx* c, const double* q0, const double* p0, const double* h,
                          const int64_t* nsteps, const int64_t* out_stride, double* q_out,
                          double* p_out, irkgl16_stats* stats) {
  if (!c) return IRKGL16_EINVAL;
  const int32_t n = c->n_inst;
  if (c->ode) {  // first-order form: y in q0 / q_out; p0 and p_out are not used
    p0 = nullptr;
    p_out = nullptr;
  }
  if (n > 0 && (!q0 || (!p0 && !c->ode) || !h || !nsteps || !out_stride || !q_out ||
                (!p_out && !c->ode)))
    return IRKGL16_EINVAL;
  int64_t out_total = 0, iters_total = 0;
  for (int32_t i = 0; i < n; ++i) {
    if (!std::isfinite(h[i]) || h[i] == 0.0 || nsteps[i] < 0 || out_stride[i] < 1 ||
        nsteps[i] % out_stride[i] != 0)
      return IRKGL16_EINVAL;
    irk::InstDesc& d = c->desc[i];
    d.h = h[i];
    d.nsteps = nsteps[i];
    d.stride = out_stride[i];
    d.out_off = out_total;
    out_total += (int64_t)c->dq[i] * (nsteps[i] / out_stride[i] + 1);
    d.iters_off = c->record ? iters_total : -1;
    iters_total += nsteps[i];
  }
  if (hipSetDevice(c->device) != hipSuccess) return IRKGL16_EDEVICE;
  const bool dev = (c->flags & IRKGL16_DEVICE_PTRS) != 0;
  const double *dq0 = q0, *dp0 = p0;
  double *dqo = q_out, *dpo = p_out;
  if (!dev) {
    ALLOC_TRY(c->d_q0, sizeof(double) * (size_t)std::max<int64_t>(c->total_dq, 1));
    ALLOC_TRY(c->d_qout, sizeof(double) * (size_t)std::max<int64_t>(out_total, 1));
    dq0 = c->d_q0.as<double>();
    dqo = c->d_qout.as<double>();
    if (!c->ode) {
      ALLOC_TRY(c->d_p0, sizeof(double) * (size_t)std::max<int64_t>(c->total_dq, 1));
      ALLOC_TRY(c->d_pout, sizeof(double) * (size_t)std::max<int64_t>(out_total, 1));
      dp0 = c->d_p0.as<double>();
      dpo = c->d_pout.as<double>();
    }
  }
  if (c->record) ALLOC_TRY(c->d_iters, (size_t)std::max<int64_t>(iters_total, 1));
  c->last_nsteps.assign(nsteps, nsteps + n);
  c->last_iters_total = iters_total;
  c->have_last = true;
  c->last_synced = false;
  if (n == 0) return IRKGL16_OK;

  // Class queues, longest integrations first (estimated work nsteps x step cost).
  c->h_queue.resize(n);
  for (auto& kc : c->classes) {
    std::vector<int32_t> ids = kc.ids;
    std::stable_sort(ids.begin(), ids.end(), [&](int32_t x, int32_t y) {
      return (double)nsteps[x] * step_work(c->desc[x]) > (double)nsteps[y] * step_work(c->desc[y]);
    });
    std::copy(ids.begin(), ids.end(), c->h_queue.begin() + kc.queue_off);
  }
  HIP_TRY(hipMemcpyAsync(c->d_queue.p, c->h_queue.data(), sizeof(int32_t) * n,
                         hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipMemcpyAsync(c->d_desc.p, c->desc.data(), sizeof(irk::InstDesc) * n,
                         hipMemcpyHostToDevice, c->stream));
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(c->d_q0.p, q0, sizeof(double) * c->total_dq, hipMemcpyHostToDevice,
                           c->stream));
    if (!c->ode)
      HIP_TRY(hipMemcpyAsync(c->d_p0.p, p0, sizeof(double) * c->total_dq, hipMemcpyHostToDevice,
                             c->stream));
  }
  HIP_TRY(hipEventRecord(c->ev0, c->stream));
  HIP_TRY(irk::launch_prepare(c->d_desc.as<irk::InstDesc>(), c->d_stat.as<irk::InstStat>(),
                              c->d_state.as<double>(), c->d_params.as<double>(), dq0, dp0, dqo,
                              dpo, c->record ? c->d_iters.as<uint8_t>() : nullptr,
                              c->d_heads.as<int32_t>(), (int)c->classes.size(), n, c->stream, nullptr,
                              c->d_prev.as<int64_t>(), c->d_evicted.as<uint8_t>()));
  irk::LaunchArgs a = base_args(c, dqo, dpo);
  if ((c->flags & IRKGL16_PLAIN) && (c->flags & IRKGL16_GRAPH)) {
    // Plain form with the step loop in a graph: one step's launches (one per
    // instance, single-step budget) captured once, replayed max(nsteps) times.
    HIP_TRY(plain_graph_steps(c, a, nsteps));
    // An instance that stopped at a non-finite value wrote NaN frames only up
    // to the end of its one-step launch; the rest are filled here.
    HIP_TRY(irk::launch_nan_fill(c->d_desc.as<irk::InstDesc>(), c->d_stat.as<irk::InstStat>(),
                                 dqo, dpo, n, c->stream));
  } else if (c->flags & IRKGL16_PLAIN) {
    // Plain form: one launch per step per instance, instances in turn.
    for (const auto& kc : c->classes) {
      for (int32_t id : kc.ids) {
        irk::LaunchArgs pa = a;
        pa.queue = c->d_plainq.as<int32_t>() + id;
        pa.queue_len = 1;
        pa.queue_head = nullptr;
        pa.step_budget = 1;
        for (int64_t s = 0; s < nsteps[id]; ++s) HIP_TRY(launch_class(c, kc, pa, 1, c->stream));
      }
    }
    HIP_TRY(irk::launch_nan_fill(c->d_desc.as<irk::InstDesc>(), c->d_stat.as<irk::InstStat>(),
                                 dqo, dpo, n, c->stream));
  } else {
    // The whole-GPU class (cooperative launches) runs alone on the main
    // stream after the others; the batched classes run concurrently, one
    // auxiliary stream per class (round robin), joined back into the stream.
    // A class that can promote instances (or every batched class when a chunk
    // count is given) runs in chunks ending at multiples of a step count (the
    // few-body kernel stops an instance early once its iterations per step
    // grow large; it catches up in the next chunk); between chunks the order
    // kernel sorts its queue by estimated remaining work and picks the
    // instances for the stage-parallel kernel (evicted ones and slow ones),
    // whose chunk runs concurrently, at the highest wave priority, on an
    // auxiliary stream that no class uses.  The promoted chunk starts with the
    // class's own (a promoted chunk queued behind a full grid of the class's
    // workgroups would wait for free wave slots), and both end before the next
    // order kernel.  Normally all chunked classes step through their chunks
    // together, forked from and joined into the main stream, where the order
    // kernels run; a large ensemble split in two halves instead runs each half
    // as a pipeline on its own stream (order kernel included), so that the
    // halves' chunk ends fall at different times.  With every auxiliary stream
    // taken by a class, nothing is
    // promoted or chunked.  An instance whose iteration slows down mid-run is
    // thus neither pulled late nor left on the slower path.  Every launch
    // resumes each instance's state exactly, so chunking never changes
    // results.  The first chunk takes the class's full member list (d_queue,
    // never written during the call); later chunks take the order kernel's
    // queues (d_queue2, d_qprom) with their lengths in device memory.
    const int32_t* members = c->d_queue.as<int32_t>();
    int32_t* qnorm = c->d_queue2.as<int32_t>();
    int32_t* counts = c->d_counts.as<int32_t>();
    const int naux = (int)c->aux.size();
    int n_batched = 0;
    for (const auto& kc : c->classes) n_batched += kc.cls != irk::kClassLarge;
    struct Plan {
      int k, j, jp, nch;  // class, its stream, promotion stream (-1: none), chunks
      int64_t budget;
    };
    // Classes in order of decreasing estimated duration, each to the stream
    // with the least estimated work so far (so the longest class starts at
    // once and on a stream of its own when there are more classes than
    // streams).
    std::vector<int> order;
    std::vector<double> est(c->classes.size(), 0.0);
    for (size_t k = 0; k < c->classes.size(); ++k) {
      if (c->classes[k].cls == irk::kClassLarge) continue;
      order.push_back((int)k);
      est[k] = class_estimate(c->classes[k], nsteps);
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return est[x] > est[y]; });
    std::vector<double> load(std::max(1, std::min(naux, n_batched)), 0.0);
    std::vector<Plan> plans;
    int prom_slot = 0, max_nch = 1;
    for (int k : order) {
      const auto& kc = c->classes[k];
      const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[j] += est[k];
      Plan pl{k, j, -1, 1, 0};
      const bool prom = promotable(c, kc) && n_batched < naux;
      if (prom) pl.jp = n_batched + prom_slot++ % (naux - n_batched);
      int64_t max_steps = 0;
      for (int32_t id : kc.ids) max_steps = std::max(max_steps, nsteps[id]);
      pl.nch = (prom || c->chunks > 0) ? chunk_count(c->chunks, max_steps, c->max_chunks) : 1;
      pl.budget = pl.nch > 1 ? (max_steps + pl.nch - 1) / pl.nch : 0;
      max_nch = std::max(max_nch, pl.nch);
      plans.push_back(pl);
    }
    if (c->halves) {
      // Each class runs its chunks as a pipeline on its own stream: chunk, then
      // (joined with its promoted chunk) the order kernel, then the next chunk.
      // Classes do not wait for each other at chunk boundaries, so one class's
      // wavefronts fill the GPU while another drains the end of a chunk.
      HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
      std::vector<char> used(c->aux.size(), 0);
      auto start = [&](int j) -> hipError_t {
        if (used[j]) return hipSuccess;
        used[j] = 1;
        return hipStreamWaitEvent(c->aux[j], c->ev_fork, 0);
      };
      for (const Plan& pl : plans) {
        const auto& kc = c->classes[pl.k];
        hipStream_t sj = c->aux[pl.j];
        HIP_TRY(start(pl.j));
        if (pl.jp >= 0) HIP_TRY(start(pl.jp));
        for (int ch = 0; ch < pl.nch; ++ch) {
          irk::LaunchArgs ca = a;
          ca.queue = (ch == 0 ? members : qnorm) + kc.queue_off;
          ca.queue_len = (int32_t)kc.ids.size();
          ca.queue_head = c->d_heads.as<int32_t>() + pl.k;
          // chunk boundary: instances behind it (evicted ones) catch up; the
          // last chunk runs every instance to its end
          ca.step_limit = (pl.nch > 1 && ch + 1 < pl.nch) ? (ch + 1) * pl.budget : 0;
          if (pl.jp >= 0 && ch + 1 < pl.nch) {
            ca.evict_k = c->evict_k;
            ca.evicted = c->d_evicted.as<uint8_t>();
          }
          if (ch > 0) ca.queue_len_dev = counts + 2 * pl.k;  // set by the order kernel
          const bool prom_chunk = ch > 0 && pl.jp >= 0;
          if (prom_chunk) {  // the promoted chunk starts with the class's chunk
            HIP_TRY(hipEventRecord(c->aux_done[pl.j], sj));
            HIP_TRY(hipStreamWaitEvent(c->aux[pl.jp], c->aux_done[pl.j], 0));
          }
          HIP_TRY(launch_class(c, kc, ca, (int)kc.ids.size(), sj));
          if (prom_chunk) {
            KernelClass ks = kc;
            ks.cls = irk::kClassStage;
            ks.size = irk::stage_np(kc.size);
            irk::LaunchArgs pa = ca;
            pa.evict_k = 0.0;
            pa.promoted = 1;
            pa.queue = c->d_qprom.as<int32_t>() + kc.queue_off;
            pa.queue_len_dev = counts + 2 * pl.k + 1;
            pa.queue_head = c->d_heads_prom.as<int32_t>() + pl.k;
            HIP_TRY(launch_class(c, ks, pa, std::min((int)kc.ids.size(), c->num_cus),
                                 c->aux[pl.jp]));
          }
          if (ch + 1 == pl.nch) break;
          // join the promoted chunk, then order the next chunk
          if (prom_chunk) {
            HIP_TRY(hipEventRecord(c->aux_done[pl.jp], c->aux[pl.jp]));
            HIP_TRY(hipStreamWaitEvent(sj, c->aux_done[pl.jp], 0));
          }
          HIP_TRY(irk::launch_order(members + kc.queue_off, qnorm + kc.queue_off,
                                    (int32_t)kc.ids.size(), c->d_desc.as<irk::InstDesc>(),
                                    c->d_stat.as<irk::InstStat>(), c->d_prev.as<int64_t>(),
                                    c->d_heads.as<int32_t>() + pl.k,
                                    c->d_qprom.as<int32_t>() + kc.queue_off, counts + 2 * pl.k,
                                    c->d_heads_prom.as<int32_t>() + pl.k,
                                    pl.jp >= 0 ? c->promote_k : 0.0,
                                    c->d_evicted.as<uint8_t>(), sj));
        }
      }
      for (int j = 0; j < naux; ++j) {
        if (!used[j]) continue;
        HIP_TRY(hipEventRecord(c->aux_done[j], c->aux[j]));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->aux_done[j], 0));
      }
    } else {
      // One class, or classes that each fit the GPU: all chunked classes step
      // through their chunks together, the order kernels on the main stream.
      std::vector<char> used(c->aux.size(), 0);
      auto fork = [&](int j) -> hipError_t {
        used[j] = 1;
        return hipStreamWaitEvent(c->aux[j], c->ev_fork, 0);
      };
      for (int ch = 0; ch < max_nch; ++ch) {
        HIP_TRY(hipEventRecord(c->ev_fork, c->stream));
        std::vector<char> step_used(c->aux.size(), 0);
        for (const Plan& pl : plans) {
          if (ch >= pl.nch || (ch > 0 && pl.nch == 1)) continue;
          const auto& kc = c->classes[pl.k];
          irk::LaunchArgs ca = a;
          ca.queue = (ch == 0 ? members : qnorm) + kc.queue_off;
          ca.queue_len = (int32_t)kc.ids.size();
          ca.queue_head = c->d_heads.as<int32_t>() + pl.k;
          // chunk boundary: instances behind it (evicted ones) catch up; the
          // last chunk runs every instance to its end
          ca.step_limit = (pl.nch > 1 && ch + 1 < pl.nch) ? (ch + 1) * pl.budget : 0;
          if (pl.jp >= 0 && ch + 1 < pl.nch) {
            ca.evict_k = c->evict_k;
            ca.evicted = c->d_evicted.as<uint8_t>();
          }
          if (ch > 0) ca.queue_len_dev = counts + 2 * pl.k;  // set by the order kernel
          HIP_TRY(fork(pl.j));
          if (pl.nch > 1) step_used[pl.j] = 1;
          HIP_TRY(launch_class(c, kc, ca, (int)kc.ids.size(), c->aux[pl.j]));
          if (ch > 0 && pl.jp >= 0) {
            KernelClass ks = kc;
            ks.cls = irk::kClassStage;
            ks.size = irk::stage_np(kc.size);
            irk::LaunchArgs pa = ca;
            pa.evict_k = 0.0;
            pa.promoted = 1;
            pa.queue = c->d_qprom.as<int32_t>() + kc.queue_off;
            pa.queue_len_dev = counts + 2 * pl.k + 1;
            pa.queue_head = c->d_heads_prom.as<int32_t>() + pl.k;
            HIP_TRY(fork(pl.jp));
            step_used[pl.jp] = 1;
            HIP_TRY(launch_class(c, ks, pa, std::min((int)kc.ids.size(), c->num_cus),
                                 c->aux[pl.jp]));
          }
        }
        if (ch + 1 == max_nch) break;
        // join the chunked classes' streams, then order their next chunk
        for (int j = 0; j < naux; ++j) {
          if (!step_used[j]) continue;
          HIP_TRY(hipEventRecord(c->aux_done[j], c->aux[j]));
          HIP_TRY(hipStreamWaitEvent(c->stream, c->aux_done[j], 0));
        }
        for (const Plan& pl : plans) {
          if (ch + 1 >= pl.nch) continue;
          const auto& kc = c->classes[pl.k];
          HIP_TRY(irk::launch_order(members + kc.queue_off, qnorm + kc.queue_off,
                                    (int32_t)kc.ids.size(), c->d_desc.as<irk::InstDesc>(),
                                    c->d_stat.as<irk::InstStat>(), c->d_prev.as<int64_t>(),
                                    c->d_heads.as<int32_t>() + pl.k,
                                    c->d_qprom.as<int32_t>() + kc.queue_off, counts + 2 * pl.k,
                                    c->d_heads_prom.as<int32_t>() + pl.k,
                                    pl.jp >= 0 ? c->promote_k : 0.0,
                                    c->d_evicted.as<uint8_t>(), c->stream));
        }
      }
      for (int j = 0; j < naux; ++j) {
        if (!used[j]) continue;
        HIP_TRY(hipEventRecord(c->aux_done[j], c->aux[j]));
        HIP_TRY(hipStreamWaitEvent(c->stream, c->aux_done[j], 0));
      }
    }
    if (max_nch > 1)
      HIP_TRY(irk::launch_nan_fill(c->d_desc.as<irk::InstDesc>(), c->d_stat.as<irk::InstStat>(),
                                   dqo, dpo, n, c->stream));
    for (size_t k = 0; k < c->classes.size(); ++k) {
      const auto& kc = c->classes[k];
      if (kc.cls != irk::kClassLarge) continue;
      irk::LaunchArgs ca = a;
      ca.queue = c->d_queue.as<int32_t>() + kc.queue_off;
      ca.queue_len = (int32_t)kc.ids.size();
      ca.queue_head = c->d_heads.as<int32_t>() + k;
      HIP_TRY(launch_class(c, kc, ca, (int)kc.ids.size(), c->stream));
    }
  }
  HIP_TRY(hipEventRecord(c->ev1, c->stream));
  if (!dev) {
    HIP_TRY(hipMemcpyAsync(q_out, dqo, sizeof(double) * out_total, hipMemcpyDeviceToHost,
                           c->stream));
    if (!c->ode)
      HIP_TRY(hipMemcpyAsync(p_out, dpo, sizeof(double) * out_total, hipMemcpyDeviceToHost,
                             c->stream));
    return irkgl16_last_stats(c, stats);
  }
  if (stats) return irkgl16_last_stats(c, stats);
  return IRKGL16_OK;
}

extern "C" {

int irkgl16_create(irkgl16_ctx** out, const irkgl16_problem* probs, int32_t n_inst,
                   const irkgl16_options* opt, void* hip_stream) {
  try {
    return create_impl(out, probs, n_inst, opt, hip_stream);
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

int irkgl16_create_user(irkgl16_ctx** out, const char* force_src, int32_t dq, int32_t n_params,
                        const double* params, int32_t n_inst, const irkgl16_options* opt,
                        void* hip_stream) {
  try {
    if (!out) return IRKGL16_EINVAL;
    *out = nullptr;
    if (n_inst < 0 || !force_src || !irk::user_dq_supported(dq)) return IRKGL16_EINVAL;
    std::vector<irkgl16_problem> probs((size_t)std::max(n_inst, 1));
    for (auto& p : probs) {
      std::memset(&p, 0, sizeof(p));
      p.kind = irk::kUser;
      p.n = 1;
      p.d = dq;
    }
    const UserSpec spec{force_src, dq, n_params, params, false};
    return create_impl(out, probs.data(), n_inst, opt, hip_stream, &spec);
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

int irkgl16_create_ode(irkgl16_ctx** out, const char* rhs_src, int32_t D, int32_t n_params,
                       const double* params, int32_t n_inst, const irkgl16_options* opt,
                       void* hip_stream) {
  try {
    if (!out) return IRKGL16_EINVAL;
    *out = nullptr;
    if (n_inst < 0 || !rhs_src || !irk::user_dq_supported(D)) return IRKGL16_EINVAL;
    std::vector<irkgl16_problem> probs((size_t)std::max(n_inst, 1));
    for (auto& p : probs) {
      std::memset(&p, 0, sizeof(p));
      p.kind = irk::kUserOde;
      p.n = 1;
      p.d = D;
    }
    const UserSpec spec{rhs_src, D, n_params, params, true};
    return create_impl(out, probs.data(), n_inst, opt, hip_stream, &spec);
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

static int compile_check(const char* src, int32_t dq, bool ode, char* log, int64_t log_len) {
  try {
    std::string l;
    const int rc = irk::user_compile_check(src, dq, ode, &l);
    if (log && log_len > 0) {
      const size_t n = std::min<size_t>(l.size(), (size_t)(log_len - 1));
      std::memcpy(log, l.data(), n);
      log[n] = '\0';
    }
    return rc == 0 ? IRKGL16_OK : IRKGL16_EINVAL;
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

int irkgl16_user_compile_check(const char* force_src, int32_t dq, char* log, int64_t log_len) {
  return compile_check(force_src, dq, false, log, log_len);
}

int irkgl16_ode_compile_check(const char* rhs_src, int32_t D, char* log, int64_t log_len) {
  return compile_check(rhs_src, D, true, log, log_len);
}

int irkgl16_integrate(irkgl16_ctx* ctx, const double* q0, const double* p0, const double* h,
                      const int64_t* nsteps, const int64_t* out_stride, double* q_out,
                      double* p_out, irkgl16_stats* stats) {
  try {
    return integrate_impl(ctx, q0, p0, h, nsteps, out_stride, q_out, p_out, stats);
  } catch (const std::bad_alloc&) {
    return IRKGL16_ENOMEM;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

int irkgl16_last_stats(irkgl16_ctx* c, irkgl16_stats* stats) {
  if (!c) return IRKGL16_EINVAL;
  if (!c->have_last) return IRKGL16_EINVAL;
  try {
    if (!c->last_synced) {
      HIP_TRY(hipStreamSynchronize(c->stream));
      c->h_stat.resize(c->n_inst);
      if (c->n_inst > 0)
        HIP_TRY(hipMemcpy(c->h_stat.data(), c->d_stat.p, sizeof(irk::InstStat) * c->n_inst,
                          hipMemcpyDeviceToHost));
      float ms = 0.f;
      if (c->n_inst > 0 && hipEventElapsedTime(&ms, c->ev0, c->ev1) == hipSuccess)
        c->last_ms = ms;
      else
        c->last_ms = 0.f;
      c->last_synced = true;
    }
    const int worst = irk::summarize_stats(c->h_stat.data(), c->n_inst, stats);
    if (stats) {
      stats->device_ms = (double)c->last_ms;
      if (stats->step_iters && c->record && c->last_iters_total > 0)
        HIP_TRY(hipMemcpy(stats->step_iters, c->d_iters.p, (size_t)c->last_iters_total,
                          hipMemcpyDeviceToHost));
    }
    return worst;
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

void irkgl16_destroy(irkgl16_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  delete ctx;
}

const char* irkgl16_strerror(int status) {
  switch (status) {
    case IRKGL16_OK: return "ok";
    case IRKGL16_EINVAL: return "invalid argument";
    case IRKGL16_ENOMEM: return "out of memory";
    case IRKGL16_EDEVICE: return "no usable gfx950 GPU or HIP runtime error";
    case IRKGL16_ENONFINITE: return "an instance produced a non-finite value";
    case IRKGL16_ENOCONV: return "some steps stopped at the iteration cap";
    case IRKGL16_ESCRATCH:
      return "the call does not fit the fixed scratch of irkgl16_integrate_static";
    case IRKGL16_ECANCELED: return "the request was cancelled";
    default: return "unknown status";
  }
}

}  // extern "C"

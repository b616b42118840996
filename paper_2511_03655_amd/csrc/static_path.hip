// Allocation-free integration: irkgl16_integrate_static.
//
// The same batched kernels as irkgl16_create + irkgl16_integrate, for callers
// that cannot allocate device memory while they integrate.  Everything a call
// needs on the device beyond the caller's inputs and outputs -- coefficient
// table, instance descriptors, masses/couplings, class queues and their
// counters, statistics, the resumable state records and (optionally) the
// per-step iteration counts -- is carved out of one fixed device array,
// `scratch`, of IRKGL16_STATIC_SCRATCH_BYTES per GPU.  Host-side staging uses
// fixed file-scope arrays as well, so a call allocates nothing on the host or
// the device.
//
// Scratch layout of a call (byte offsets, each region 256-byte aligned):
//   [table | descriptors | parameters | queue]   uploaded from the host stage
//   [statistics | queue counters | state records | iteration counts]
//                                                written by the setup kernel
// The upload part has the same layout in the host stage, so it goes to the
// device in one copy.
//
// Set-up, once per device on the first call there (with that device
// current): the device address of `scratch` (hipGetSymbolAddress; in host
// code the array's name is only a stand-in, never a device address), and
// three events (the host stage is rewritten only after the previous call's
// upload has finished; the call's device time).  Every call on a GPU reuses
// that GPU's scratch: calls are serialized on the host by a mutex, and calls
// enqueued on different streams of one GPU without synchronization race on
// the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "../../include/irkgl16.h"
#include "device_common.h"
#include "host_common.h"
#include "launch.h"

// One copy per GPU, held until the process ends.
static __device__ __align__(256) unsigned char scratch[IRKGL16_STATIC_SCRATCH_BYTES];

namespace {

constexpr int64_t kScratchBytes = IRKGL16_STATIC_SCRATCH_BYTES;
constexpr int kMaxInst = IRKGL16_STATIC_MAX_INST;
constexpr int64_t kStageBytes = 4ll << 20;  // host stage: table, descriptors, parameters, queue
constexpr int kMaxClasses = 64;
constexpr int kMaxDevices = 64;
constexpr int64_t kAlign = 256;

struct DeviceSetup {
  bool ready = false;
  unsigned char* ptr = nullptr;  // device address of `scratch` on this GPU
  int num_cus = 1;
  hipEvent_t uploaded = nullptr;  // the last call's upload has read the host stage
  bool upload_pending = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // device time of the last call
};

struct ClassSlot {
  int cls, kind, size, d;
  int32_t count;
  int64_t queue_off;  // first queue entry of the class
};

alignas(256) unsigned char g_stage[kStageBytes];
irk::InstStat g_hstat[kMaxInst];
int32_t g_class_of[kMaxInst];
ClassSlot g_classes[kMaxClasses];
DeviceSetup g_dev[kMaxDevices];
std::mutex g_mutex;

int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Looks up the scratch address and creates the events of the current device.
int device_setup(int dev, DeviceSetup** out) {
  DeviceSetup& s = g_dev[dev];
  if (!s.ready) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return IRKGL16_EDEVICE;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return IRKGL16_EDEVICE;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr)
      return IRKGL16_EDEVICE;
    if (hipEventCreateWithFlags(&s.uploaded, hipEventDisableTiming) != hipSuccess ||
        hipEventCreate(&s.ev0) != hipSuccess || hipEventCreate(&s.ev1) != hipSuccess)
      return IRKGL16_EDEVICE;
    s.ptr = static_cast<unsigned char*>(p);
    s.num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 1;
    s.ready = true;
  }
  *out = &s;
  return IRKGL16_OK;
}

double step_work(const irk::InstDesc& d) {
  const double n = d.n;
  return d.kind == IRKGL16_GRAVITY ? n * n * d.d : n * d.d;
}

#define HIP_TRY(expr)                             \
  do {                                            \
    if ((expr) != hipSuccess) return IRKGL16_EDEVICE; \
  } while (0)

int integrate_static_impl(const irkgl16_problem* probs, int32_t n, const irkgl16_options* opt,
                          void* hip_stream, const double* q0, const double* p0, const double* h,
                          const int64_t* nsteps, const int64_t* out_stride, double* q_out,
                          double* p_out, irkgl16_stats* stats) {
  // ---- arguments (host only, before any device call)
  if (n < 0 || (n > 0 && (!probs || !q0 || !p0 || !h || !nsteps || !out_stride || !q_out ||
                          !p_out)))
    return IRKGL16_EINVAL;
  const uint32_t flags = opt ? opt->flags : 0u;
  if (flags & ~(IRKGL16_DEVICE_PTRS | IRKGL16_REPRODUCIBLE)) return IRKGL16_EINVAL;
  if (opt && ((opt->stages != 0 && opt->stages != irk::kS) || opt->method != 0))
    return IRKGL16_EINVAL;
  const bool record = opt && opt->record_iters != 0;
  int32_t max_iter = (opt && opt->max_iter > 0) ? opt->max_iter : 100;
  if (record && max_iter > 255) max_iter = 255;  // counts stored as bytes
  if (n > kMaxInst) return IRKGL16_ESCRATCH;

  int64_t n_params = 0, state_doubles = 0, iters_total = 0, out_total = 0, total_dq = 0;
  int n_classes = 0;
  for (int32_t i = 0; i < n; ++i) {
    const irkgl16_problem& p = probs[i];
    if (irk::validate_problem(p) != IRKGL16_OK) return IRKGL16_EINVAL;
    int size = 0;
    const int cl = irk::kernel_class(p.kind, p.n, p.d, &size);
    // The whole-GPU class keeps grid-barrier state of its own; not served here.
    if (cl < 0 || cl == irk::kClassLarge) return IRKGL16_EINVAL;
    if (!std::isfinite(h[i]) || h[i] == 0.0 || nsteps[i] < 0 || out_stride[i] < 1 ||
        nsteps[i] % out_stride[i] != 0)
      return IRKGL16_EINVAL;
    int k = 0;
    while (k < n_classes && !(g_classes[k].cls == cl && g_classes[k].kind == p.kind &&
                              g_classes[k].size == size && g_classes[k].d == p.d))
      ++k;
    if (k == n_classes) {
      if (n_classes == kMaxClasses) return IRKGL16_ESCRATCH;
      g_classes[n_classes++] = ClassSlot{cl, p.kind, size, p.d, 0, 0};
    }
    ++g_classes[k].count;
    g_class_of[i] = k;
    const int64_t dq = (int64_t)p.n * p.d;
    if (p.mass && p.kind != IRKGL16_KEPLER) n_params += p.n;
    if (p.coupling && p.kind == IRKGL16_CHAIN) n_params += p.n + 1;
    state_doubles += (4 + irk::kS) * dq;
    total_dq += dq;
    out_total += dq * (nsteps[i] / out_stride[i] + 1);
    iters_total += nsteps[i];
  }

  // ---- layout and size checks
  const int64_t off_tab = 0;
  const int64_t off_desc = align_up(off_tab + (int64_t)sizeof(double) * irk::kTabSize);
  const int64_t off_params = align_up(off_desc + (int64_t)sizeof(irk::InstDesc) * n);
  const int64_t off_queue = align_up(off_params + (int64_t)sizeof(double) * n_params);
  const int64_t upload_bytes = off_queue + (int64_t)sizeof(int32_t) * n;
  const int64_t off_stat = align_up(upload_bytes);
  const int64_t off_heads = align_up(off_stat + (int64_t)sizeof(irk::InstStat) * n);
  const int64_t off_state = align_up(off_heads + (int64_t)sizeof(int32_t) * n_classes);
  const int64_t off_iters = align_up(off_state + (int64_t)sizeof(double) * state_doubles);
  const int64_t total_bytes = off_iters + (record ? iters_total : 0);
  if (upload_bytes > kStageBytes || total_bytes > kScratchBytes) return IRKGL16_ESCRATCH;

  if (stats) {
    stats->steps = stats->iterations = stats->nonconverged_steps = 0;
    stats->max_k = stats->n_nonfinite = 0;
    stats->device_ms = 0.0;
  }
  if (n == 0) return IRKGL16_OK;

  // ---- device set-up (first call on this GPU)
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return IRKGL16_EDEVICE;
  DeviceSetup* ds = nullptr;
  if (int rc = device_setup(dev, &ds)) return rc;
  hipStream_t stream = (hipStream_t)hip_stream;

  // ---- host stage: the previous call's upload must have read it
  if (ds->upload_pending) {
    HIP_TRY(hipEventSynchronize(ds->uploaded));
    ds->upload_pending = false;
  }
  unsigned char* S = g_stage;
  std::memcpy(S + off_tab, irk::kTabS8, sizeof(double) * irk::kTabSize);
  irk::InstDesc* desc = reinterpret_cast<irk::InstDesc*>(S + off_desc);
  double* params = reinterpret_cast<double*>(S + off_params);
  int32_t* queue = reinterpret_cast<int32_t*>(S + off_queue);
  {
    int64_t po = 0, so = 0, io = 0, oo = 0, in = 0;
    for (int32_t i = 0; i < n; ++i) {
      const irkgl16_problem& p = probs[i];
      irk::InstDesc& d = desc[i];
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
        d.mass_off = po;
        std::memcpy(params + po, p.mass, sizeof(double) * p.n);
        po += p.n;
      }
      if (p.coupling && p.kind == IRKGL16_CHAIN) {
        d.coupling_off = po;
        std::memcpy(params + po, p.coupling, sizeof(double) * (p.n + 1));
        po += p.n + 1;
      }
      const int64_t dq = (int64_t)p.n * p.d;
      d.in_off = in;
      in += dq;
      d.state_off = so;
      so += (4 + irk::kS) * dq;
      d.h = h[i];
      d.nsteps = nsteps[i];
      d.stride = out_stride[i];
      d.out_off = oo;
      oo += dq * (nsteps[i] / out_stride[i] + 1);
      d.iters_off = record ? io : -1;
      io += nsteps[i];
    }
  }
  // class queues, longest integrations first (order never changes results)
  {
    int64_t off = 0;
    for (int k = 0; k < n_classes; ++k) {
      g_classes[k].queue_off = off;
      off += g_classes[k].count;
      g_classes[k].count = 0;
    }
    for (int32_t i = 0; i < n; ++i) {
      ClassSlot& c = g_classes[g_class_of[i]];
      queue[c.queue_off + c.count++] = i;
    }
    for (int k = 0; k < n_classes; ++k) {
      int32_t* b = queue + g_classes[k].queue_off;
      std::sort(b, b + g_classes[k].count, [&](int32_t x, int32_t y) {
        const double wx = (double)desc[x].nsteps * step_work(desc[x]);
        const double wy = (double)desc[y].nsteps * step_work(desc[y]);
        return wx > wy || (wx == wy && x < y);
      });
    }
  }

  // ---- enqueue: upload, setup kernel, one persistent launch per class
  unsigned char* D = ds->ptr;
  const double* d_tab = reinterpret_cast<const double*>(D + off_tab);
  irk::InstDesc* d_desc = reinterpret_cast<irk::InstDesc*>(D + off_desc);
  double* d_params = reinterpret_cast<double*>(D + off_params);
  int32_t* d_queue = reinterpret_cast<int32_t*>(D + off_queue);
  irk::InstStat* d_stat = reinterpret_cast<irk::InstStat*>(D + off_stat);
  int32_t* d_heads = reinterpret_cast<int32_t*>(D + off_heads);
  double* d_state = reinterpret_cast<double*>(D + off_state);
  uint8_t* d_iters = record ? reinterpret_cast<uint8_t*>(D + off_iters) : nullptr;

  HIP_TRY(hipMemcpyAsync(D, S, (size_t)upload_bytes, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipEventRecord(ds->uploaded, stream));
  ds->upload_pending = true;
  HIP_TRY(hipEventRecord(ds->ev0, stream));
  HIP_TRY(irk::launch_prepare(d_desc, d_stat, d_state, d_params, q0, p0, q_out, p_out, d_iters,
                              d_heads, n_classes, n, stream));
  for (int k = 0; k < n_classes; ++k) {
    const ClassSlot& c = g_classes[k];
    irk::LaunchArgs a;
    a.tab = d_tab;
    a.desc = d_desc;
    a.stat = d_stat;
    a.state = d_state;
    a.params = d_params;
    a.qout = q_out;
    a.pout = p_out;
    a.step_iters = d_iters;
    a.queue = d_queue + c.queue_off;
    a.queue_len = c.count;
    a.max_iter = max_iter;
    a.queue_head = d_heads + k;
    a.step_budget = 0;
    a.exact = (flags & IRKGL16_REPRODUCIBLE) ? 1 : 0;
    HIP_TRY(irk::launch_batched(c.cls, c.kind, c.size, c.d, a, c.count, ds->num_cus, stream));
  }
  HIP_TRY(hipEventRecord(ds->ev1, stream));
  if (!stats) return IRKGL16_OK;

  // ---- statistics (synchronizes the stream)
  HIP_TRY(hipMemcpyAsync(g_hstat, d_stat, sizeof(irk::InstStat) * n, hipMemcpyDeviceToHost,
                         stream));
  if (stats->step_iters && record && iters_total > 0)
    HIP_TRY(hipMemcpyAsync(stats->step_iters, d_iters, (size_t)iters_total, hipMemcpyDeviceToHost,
                           stream));
  HIP_TRY(hipStreamSynchronize(stream));
  ds->upload_pending = false;
  const int worst = irk::summarize_stats(g_hstat, n, stats);
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, ds->ev0, ds->ev1) == hipSuccess) stats->device_ms = (double)ms;
  return worst;
}

}  // namespace

extern "C" int irkgl16_integrate_static(const irkgl16_problem* probs, int32_t n_inst,
                                        const irkgl16_options* opt, void* hip_stream,
                                        const double* q0, const double* p0, const double* h,
                                        const int64_t* nsteps, const int64_t* out_stride,
                                        double* q_out, double* p_out, irkgl16_stats* stats) {
  try {
    std::lock_guard<std::mutex> lock(g_mutex);
    return integrate_static_impl(probs, n_inst, opt, hip_stream, q0, p0, h, nsteps, out_stride,
                                 q_out, p_out, stats);
  } catch (...) {
    return IRKGL16_EDEVICE;
  }
}

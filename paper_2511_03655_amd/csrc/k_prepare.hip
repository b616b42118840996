// Per-call setup kernel (one block per instance; `ids`, if given, lists the
// instances to set up; p0 and pout are null for first-order contexts, whose
// state is y = q0 alone): converts the caller's initial (q0, p0) into the
// resumable device state (q and v = fl(p / m) as two-double values with zero
// low parts, previous-step increments R_prev = 0 so that the first initial
// guess uses the current velocity only), writes output frame 0 (q, m v), clears
// per-instance statistics and iteration records, and zeroes the work-queue
// counters used by the integration kernels.
#include "device_common.h"

namespace irk {

__global__ __launch_bounds__(64) void prepare_kernel(const InstDesc* __restrict__ desc,
                                                     InstStat* __restrict__ stat,
                                                     double* __restrict__ state,
                                                     const double* __restrict__ params,
                                                     const double* __restrict__ q0,
                                                     const double* __restrict__ p0,
                                                     double* __restrict__ qout,
                                                     double* __restrict__ pout,
                                                     uint8_t* __restrict__ step_iters,
                                                     int32_t* __restrict__ heads, int n_heads,
                                                     const int32_t* __restrict__ ids,
                                                     int64_t* __restrict__ prev,
                                                     uint8_t* __restrict__ evicted) {
  const int i = ids ? ids[blockIdx.x] : (int)blockIdx.x;
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < n_heads; t += blockDim.x) heads[t] = 0;
  }
  const InstDesc d = desc[i];
  const int dq = d.n * d.d;
  double* S = state + d.state_off;
  for (int c = threadIdx.x; c < dq; c += blockDim.x) {
    const double m = (d.mass_off >= 0) ? params[d.mass_off + c / d.d] : 1.0;
    const double q = q0[d.in_off + c];
    const double v = p0 ? p0[d.in_off + c] / m : 0.0;  // first-order form: no p
    S[c] = q;
    S[dq + c] = 0.0;
    S[2 * dq + c] = v;
    S[3 * dq + c] = 0.0;
    for (int s = 0; s < kS; ++s) S[4 * dq + c * kS + s] = 0.0;
    qout[d.out_off + c] = q;
    if (pout) pout[d.out_off + c] = m * v;
  }
  if (d.iters_off >= 0) {
    for (int64_t j = threadIdx.x; j < d.nsteps; j += blockDim.x) step_iters[d.iters_off + j] = 0;
  }
  if (threadIdx.x == 0) {
    InstStat st;
    st.steps_done = 0;
    st.iterations = 0;
    st.nonconv = 0;
    st.max_k = 0;
    st.status = kOk;
    stat[i] = st;
    if (prev) prev[2 * i] = prev[2 * i + 1] = 0;
    if (evicted) evicted[i] = 0;
  }
}

hipError_t launch_prepare(const InstDesc* desc, InstStat* stat, double* state,
                          const double* params, const double* q0, const double* p0, double* qout,
                          double* pout, uint8_t* step_iters, int32_t* heads, int n_heads,
                          int n_inst, hipStream_t st, const int32_t* ids, int64_t* prev,
                          uint8_t* evicted) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(prepare_kernel, dim3(n_inst), dim3(64), 0, st, desc, stat, state, params, q0,
                     p0, qout, pout, step_iters, heads, n_heads, ids, prev, evicted);
  return hipGetLastError();
}

// Queue order for the next chunk of a call that runs in chunks (a step budget
// per launch): one workgroup orders a class's members (qin: all of them, every
// time) by each instance's
// estimated remaining work -- steps left times the fixed-point iterations per
// step it needed in the chunk just run -- largest first, in buckets of half
// an octave.  Instances with nothing left go last.  The order inside a
// bucket is arbitrary: it decides only when an instance runs, never its
// arithmetic.  With promote_k > 0, instances that needed at least promote_k
// iterations per step, or that the small-system kernel evicted (evicted[id],
// cleared here), go to a second queue instead (served by a kernel with
// more lanes per instance and a shorter iteration; both kernels compute the
// same arithmetic).  counts[0], counts[1]: lengths of the two queues.
// Records each instance's counters for the next chunk and resets both queue
// heads.
constexpr int kOrderBuckets = 64;

__global__ __launch_bounds__(1024) void order_kernel(const int32_t* __restrict__ qin,
                                                     int32_t* __restrict__ qout, int32_t count,
                                                     const InstDesc* __restrict__ desc,
                                                     const InstStat* __restrict__ stat,
                                                     int64_t* __restrict__ prev,
                                                     int32_t* __restrict__ head,
                                                     int32_t* __restrict__ qprom,
                                                     int32_t* __restrict__ counts,
                                                     int32_t* __restrict__ head_prom,
                                                     double promote_k,
                                                     uint8_t* __restrict__ evicted) {
  __shared__ int32_t hist[kOrderBuckets];
  __shared__ int32_t base[kOrderBuckets];
  __shared__ int32_t nprom;
  const int tid = threadIdx.x;
  for (int b = tid; b < kOrderBuckets; b += blockDim.x) hist[b] = 0;
  if (tid == 0) nprom = 0;
  __syncthreads();
  // bucket of an instance, or -1: promoted
  auto bucket = [&](int32_t id) -> int {
    const InstStat s = stat[id];
    const int64_t rem = (s.status == kOk) ? desc[id].nsteps - s.steps_done : 0;
    if (rem <= 0) return kOrderBuckets - 1;
    const int64_t it = s.iterations - prev[2 * id], st = s.steps_done - prev[2 * id + 1];
    if (promote_k > 0.0 && evicted[id]) return -1;
    if (promote_k > 0.0 && st > 0 && (double)it >= promote_k * (double)st) return -1;
    const double kbar = st > 0 ? (double)it / (double)st : 2.0;
    int b = (int)(2.0 * log2((double)rem * (kbar > 1.0 ? kbar : 1.0)));
    b = b < 0 ? 0 : (b > kOrderBuckets - 2 ? kOrderBuckets - 2 : b);
    return kOrderBuckets - 2 - b;
  };
  for (int p = tid; p < count; p += blockDim.x) {
    const int b = bucket(qin[p]);
    if (b >= 0) atomicAdd(&hist[b], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int32_t acc = 0;
    for (int b = 0; b < kOrderBuckets; ++b) {
      base[b] = acc;
      acc += hist[b];
    }
    counts[0] = acc;
  }
  __syncthreads();
  // Each position (hence each instance) belongs to one thread, which reads the
  // old counters for its bucket before replacing them.
  for (int p = tid; p < count; p += blockDim.x) {
    const int32_t id = qin[p];
    const int b = bucket(id);
    if (b >= 0)
      qout[atomicAdd(&base[b], 1)] = id;
    else
      qprom[atomicAdd(&nprom, 1)] = id;
    prev[2 * id] = stat[id].iterations;
    prev[2 * id + 1] = stat[id].steps_done;
    evicted[id] = 0;
  }
  __syncthreads();
  if (tid == 0) {
    counts[1] = nprom;
    *head = 0;
    *head_prom = 0;
  }
}

hipError_t launch_order(const int32_t* qin, int32_t* qout, int32_t count, const InstDesc* desc,
                        const InstStat* stat, int64_t* prev, int32_t* head, int32_t* qprom,
                        int32_t* counts, int32_t* head_prom, double promote_k,
                        uint8_t* evicted, hipStream_t st) {
  hipLaunchKernelGGL(order_kernel, dim3(1), dim3(1024), 0, st, qin, qout, count, desc, stat, prev,
                     head, qprom, counts, head_prom, promote_k, evicted);
  return hipGetLastError();
}

// End of a call run in chunks: an instance that stopped at a non-finite state
// had NaN written only up to the end of the launch in which it stopped; this
// fills its remaining output frames up to the call's step count.
__global__ __launch_bounds__(64) void nan_fill_kernel(const InstDesc* __restrict__ desc,
                                                      const InstStat* __restrict__ stat,
                                                      double* __restrict__ qout,
                                                      double* __restrict__ pout) {
  const int i = blockIdx.x;
  const InstStat st = stat[i];
  if (st.status != kNonFinite) return;
  const InstDesc d = desc[i];
  const int dq = d.n * d.d;
  const int64_t f0 = first_nan_frame(st.steps_done, d.stride);
  const int64_t f1 = last_frame_of_launch(d.nsteps, d.stride);
  for (int64_t e = threadIdx.x; e < (f1 - f0 + 1) * dq; e += blockDim.x) {
    const int64_t o = frame_index(d.out_off, f0, dq, 0) + e;
    qout[o] = __builtin_nan("");
    if (pout) pout[o] = __builtin_nan("");
  }
}

hipError_t launch_nan_fill(const InstDesc* desc, const InstStat* stat, double* qout, double* pout,
                           int n_inst, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(nan_fill_kernel, dim3(n_inst), dim3(64), 0, st, desc, stat, qout, pout);
  return hipGetLastError();
}

}  // namespace irk

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
                                                     const int32_t* __restrict__ ids) {
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
  }
}

hipError_t launch_prepare(const InstDesc* desc, InstStat* stat, double* state,
                          const double* params, const double* q0, const double* p0, double* qout,
                          double* pout, uint8_t* step_iters, int32_t* heads, int n_heads,
                          int n_inst, hipStream_t st, const int32_t* ids) {
  if (n_inst <= 0) return hipSuccess;
  hipLaunchKernelGGL(prepare_kernel, dim3(n_inst), dim3(64), 0, st, desc, stat, state, params, q0,
                     p0, qout, pout, step_iters, heads, n_heads, ids);
  return hipGetLastError();
}

}  // namespace irk

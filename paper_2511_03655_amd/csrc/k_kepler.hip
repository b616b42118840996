// Latency kernel for small batches of Kepler orbits (q'' = -G q / |q|^3,
// d = 2 or 3): one 8-lane wavefront per instance, lane s = stage s.
//
// The few-body kernel runs Kepler orbits eight to a wavefront, with every
// fixed-point iteration passing through an LDS tile between a stage role and
// a component role and through the slot bookkeeping that keeps eight
// independent systems in step.  A lone orbit (a batch of a few) pays all of
// that on its critical path.  Here each lane holds its own stage: the force
// (eq. Gi) is lane-local, the 8 increments R_j reach every lane by shuffles,
// the stage update (eq. IRK_FP2) uses the lane's eta row held in registers,
// the max-norm increment (eq. Delta_n) is a DPP maximum over the 8 lanes and
// the stopping rule (eq. stopping), the compensated update (eq. qnvn2) and the
// next initial guess (eq. IRK_init2) run redundantly (update) or per stage
// (guess) in the lanes.  Every operation is the few-body kernel's own, in the
// same order (kepler_increment, stage_value, step_sums / dw_add, guess_stage),
// so an orbit gives the same bits in either kernel and the choice between them
// can depend on the batch.
#include "device_common.h"
#include "launch.h"
#include "store_index.h"

namespace irk {

// Maximum over the 8 stage lanes (DPP: swap neighbours, swap pairs, mirror
// within the 8 lanes); exact in any order.  fmax drops NaN: non-finite values
// are detected separately.
__device__ __forceinline__ double kp_group_max(double x) {
  x = fmax(x, dpp_double<0xB1>(x));
  x = fmax(x, dpp_double<0x4E>(x));
  return fmax(x, dpp_double<0x141>(x));
}

// q + h (c v + sum_j M_j R_j) with the row M and c of this lane's stage in
// registers: the operations of stage_value<false> in the same order.
__device__ __forceinline__ double kp_row_value(const double (&row)[kS], double c, double q,
                                               double v, double h, const double (&R)[kS]) {
  double acc = c * v;
#pragma unroll
  for (int j = 0; j < kS; ++j) acc = fma(row[j], R[j], acc);
  return fma(h, acc, q);
}

template <int D, bool EXACT>
__global__ __launch_bounds__(kS) void kepler_lane_kernel(LaunchArgs a) {
  const int s = threadIdx.x;  // stage
  const ConstTab T = const_tab(a.tab);

  // instance of this wavefront
  int idx = (int)blockIdx.x;
  if (a.queue_head) {
    int got = 0;
    if (s == 0) got = atomicAdd(a.queue_head, 1);
    idx = __shfl(got, 0, kS);
  }
  if (idx >= queue_length(a)) return;
  const int inst = a.queue[idx];
  const InstDesc& dsc = a.desc[inst];
  const InstStat st0 = a.stat[inst];
  const double h = dsc.h, G = dsc.G;
  const int64_t stride = dsc.stride, out_off = dsc.out_off, iters_off = dsc.iters_off;
  const int64_t state_off = dsc.state_off;
  int64_t step = st0.steps_done;
  const int64_t target = launch_target(a, step, dsc.nsteps, st0.status);
  int64_t it_sum = st0.iterations, nonconv = st0.nonconv;
  int32_t maxk = st0.max_k;
  int32_t status = st0.status;
  const double m = (dsc.mass_off >= 0) ? a.params[dsc.mass_off] : 1.0;
  const double hb = h * T[kTabB + s];
  // the fast mode's rows of this lane's stage (eta for the iteration, the
  // folded K for the initial guess)
  double eta[kS], kg[kS];
#pragma unroll
  for (int j = 0; j < kS; ++j) {
    eta[j] = a.tab[kTabEta + s * kS + j];
    kg[j] = a.tab[kTabK + s * kS + j];
  }
  const double cs = a.tab[kTabC + s];
  auto guess = [&](double q, double v, const double (&Rp)[kS]) {
    if constexpr (EXACT)
      return guess_stage<kKepler, true>(T, s, q, v, Rp, h);
    else
      return kp_row_value(kg, cs, q, v, h, Rp);
  };

  double qh[D], ql[D], vh[D], vl[D], Q[D], R[D], Rall[D][kS];
  if (step < target) {
    // state and this lane's stage of the initial guess
#pragma unroll
    for (int d = 0; d < D; ++d) {
      qh[d] = a.state[state_index(state_off, D, 0, d)];
      ql[d] = a.state[state_index(state_off, D, 1, d)];
      vh[d] = a.state[state_index(state_off, D, 2, d)];
      vl[d] = a.state[state_index(state_off, D, 3, d)];
#pragma unroll
      for (int j = 0; j < kS; ++j) Rall[d][j] = a.state[rprev_index(state_off, D, d, j, kS)];
      Q[d] = guess(qh[d], vh[d], Rall[d]);
      R[d] = Rall[d][s];
    }
  }

  while (step < target) {
    double mind[D], prv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) mind[d] = prv[d] = __builtin_inf();
    int k = 0;
    bool ok = false, bad = false;
    for (;;) {
      ++k;
      kepler_increment<D, EXACT>(Q, hb, G, R);
#pragma unroll
      for (int d = 0; d < D; ++d)
#pragma unroll
        for (int j = 0; j < kS; ++j) Rall[d][j] = __shfl(R[d], j, kS);
      ok = true;
      bool nf = false;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const double qn = EXACT ? stage_value<true>(T, s, qh[d], vh[d], h, Rall[d])
                                : kp_row_value(eta, cs, qh[d], vh[d], h, Rall[d]);
        const double dd = fabs(qn - Q[d]);
        nf |= !finite(dd);
        const double dmax = kp_group_max(dd);
        Q[d] = qn;
        ok &= stop_component(dmax, mind[d], prv[d]);
      }
      bad = __ballot(nf) != 0;
      if (bad || ok || k >= a.max_iter) break;
    }
    if (bad) {  // non-finite: this launch's remaining frames NaN, the instance stops
      if (s == 0) {
        const int64_t nfr = last_frame_of_launch(target, stride);
        for (int64_t f = first_nan_frame(step, stride); f <= nfr; ++f)
#pragma unroll
          for (int d = 0; d < D; ++d) {
            a.qout[frame_index(out_off, f, D, d)] = __builtin_nan("");
            a.pout[frame_index(out_off, f, D, d)] = __builtin_nan("");
          }
        if (iters_off >= 0) a.step_iters[iters_index(iters_off, step)] = (uint8_t)k;
      }
      status = kNonFinite;
      break;
    }
    if (s == 0 && iters_off >= 0) a.step_iters[iters_index(iters_off, step)] = (uint8_t)k;
    ++step;
    it_sum += k;
    nonconv += ok ? 0 : 1;
    maxk = k > maxk ? k : maxk;
    const bool frame = (step % stride) == 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      form_update<kKepler, EXACT>(row_tab(T), Rall[d], h, qh[d], ql[d], vh[d], vl[d]);
      if (s == 0 && frame) {
        const int64_t f = step / stride;
        a.qout[frame_index(out_off, f, D, d)] = qh[d];
        a.pout[frame_index(out_off, f, D, d)] = m * vh[d];
      }
      if (step < target) Q[d] = guess(qh[d], vh[d], Rall[d]);
    }
  }

  if (step > st0.steps_done && status == kOk) {  // resumable state for a later launch
#pragma unroll
    for (int d = 0; d < D; ++d) {
      if (s == 0) {
        a.state[state_index(state_off, D, 0, d)] = qh[d];
        a.state[state_index(state_off, D, 1, d)] = ql[d];
        a.state[state_index(state_off, D, 2, d)] = vh[d];
        a.state[state_index(state_off, D, 3, d)] = vl[d];
      }
      a.state[rprev_index(state_off, D, d, s, kS)] = R[d];
    }
  }
  if (s == 0) {
    InstStat st;
    st.steps_done = step;
    st.iterations = it_sum;
    st.nonconv = nonconv;
    st.max_k = maxk;
    st.status = status;
    a.stat[inst] = st;
  }
}

// Batches of at most this many Kepler orbits take the latency kernel.
constexpr int kKeplerLaneMaxBatch = 64;

bool kepler_lane_supported(int d, int n_items, const LaunchArgs& a) {
  return (d == 2 || d == 3) && n_items <= kKeplerLaneMaxBatch && a.evict_k <= 0.0;
}

hipError_t launch_kepler_lanes(int d, const LaunchArgs& a, int n_items, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  const bool ex = a.exact != 0;
  if (d == 2) {
    auto kern = ex ? kepler_lane_kernel<2, true> : kepler_lane_kernel<2, false>;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(kS), 0, st, a);
  } else if (d == 3) {
    auto kern = ex ? kepler_lane_kernel<3, true> : kepler_lane_kernel<3, false>;
    hipLaunchKernelGGL(kern, dim3(n_items), dim3(kS), 0, st, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace irk

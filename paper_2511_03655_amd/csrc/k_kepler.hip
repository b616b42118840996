// Latency kernel for small batches of Kepler orbits (q'' = -G q / |q|^3,
// d = 2 or 3): one 8-lane wavefront per instance, lane s = stage s.
//
// The few-body kernel runs Kepler orbits eight to a wavefront, with every
// fixed-point iteration passing through an LDS tile between a stage role and
// a component role and through the slot bookkeeping that keeps eight
// independent systems in step.  A lone orbit (a batch of a few) pays all of
// that on its critical path.  Here each lane holds its own stage:
//  * the force (eq. Gi) is lane-local;
//  * the 8 increments R_j reach every lane through a small LDS tile (each lane
//    stores its D values, then reads all 8 D), ordered by the wavefront's
//    in-order LDS pipeline rather than a barrier;
//  * the stage update (eq. IRK_FP2) uses the lane's eta row in registers;
//  * the max-norm increment (eq. Delta_n) is a DPP maximum over the 8 lanes;
//    the stopping rule (eq. stopping) cannot stop on a nonzero norm before
//    the third iteration, so the first two iterations are tested with one
//    ballot (all increments exactly zero?) and their norms are reduced only
//    when a step needs a third (most steps end at the second);
//  * the compensated update (eq. qnvn2) runs redundantly in every lane and
//    the next initial guess (eq. IRK_init2) per stage.
// Every operation is the few-body kernel's own, in the same order
// (kepler_increment, stage_value, step_sums / dw_add, guess_stage), and every
// stopping decision is the same, so an orbit gives the same bits in either
// kernel and the choice between them can depend on the batch.  The instance's
// bookkeeping is wave-uniform (scalar registers), and the frame number
// advances by counting steps instead of a 64-bit division per step.
#include "device_common.h"
#include "launch.h"
#include "store_index.h"

namespace irk {

// A double from another lane of the 8-lane group by a DPP pattern (0xB1: lane
// xor 1, 0x4E: lane xor 2, 0x141: mirror within the 8 lanes).  All 8 lanes of
// the group are active and every pattern stays inside the group, so no lane
// reads an inactive source.
template <int CTRL>
__device__ __forceinline__ double kp_dpp(double x) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}

// Orders the LDS accesses of the lanes of this one-wavefront workgroup: a
// wavefront's LDS operations execute in program order, so fences at wavefront
// scope (which emit no wait) and the wave barrier only keep the compiler from
// moving accesses across this point.
__device__ __forceinline__ void kp_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Maximum of each component's value over the 8 stage lanes, the levels of
// the components interleaved (exact in any order; fmax drops NaN, which the
// caller detects separately).
template <int D>
__device__ __forceinline__ void kp_group_max(double (&x)[D]) {
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = fmax(x[d], kp_dpp<0xB1>(x[d]));
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = fmax(x[d], kp_dpp<0x4E>(x[d]));
#pragma unroll
  for (int d = 0; d < D; ++d) x[d] = fmax(x[d], kp_dpp<0x141>(x[d]));
}

template <int D, bool EXACT>
__global__ __launch_bounds__(kS) void kepler_lane_kernel(LaunchArgs a) {
  const int s = threadIdx.x;  // stage
  const ConstTab T = const_tab(a.tab);
  // this iteration's increments, [stage][component]
  __shared__ __align__(16) double xr[kS * D];

  // instance of this wavefront (wave-uniform: its bookkeeping lives in
  // scalar registers)
  int idx = (int)blockIdx.x;
  if (a.queue_head) {
    int got = 0;
    if (s == 0) got = atomicAdd(a.queue_head, 1);
    idx = __builtin_amdgcn_readfirstlane(got);
  }
  if (idx >= queue_length(a)) return;
  const int inst = __builtin_amdgcn_readfirstlane(a.queue[idx]);
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
  // next frame by counting steps (one division per launch instead of one per step)
  FrameClock fclk = frame_clock(step, stride);
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
  // all nodes c_j (wave-uniform) for the end-of-step sums
  double cn[kS];
#pragma unroll
  for (int j = 0; j < kS; ++j) cn[j] = T[kTabC + j];

  double qh[D], ql[D], vh[D], vl[D], Q[D], R[D], Rall[D][kS];
  // stage value of every component from the rows of this lane's stage: the
  // operations of stage_value<false> (M = eta) or of the folded guess (M = K),
  // with the components' chains interleaved
  auto rows_value = [&](const double (&row)[kS], const double (&Rj)[D][kS], double (&out)[D]) {
    double acc[D];
#pragma unroll
    for (int d = 0; d < D; ++d) acc[d] = cs * vh[d];
#pragma unroll
    for (int j = 0; j < kS; ++j)
#pragma unroll
      for (int d = 0; d < D; ++d) acc[d] = fma(row[j], Rj[d][j], acc[d]);
#pragma unroll
    for (int d = 0; d < D; ++d) out[d] = fma(h, acc[d], qh[d]);
  };
  auto guess = [&]() {
    if constexpr (EXACT) {
#pragma unroll
      for (int d = 0; d < D; ++d) Q[d] = guess_stage<kKepler, true>(T, s, qh[d], vh[d], Rall[d], h);
    } else {
      rows_value(kg, Rall, Q);
    }
  };

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
      R[d] = 0.0;  // set by every iteration; stored only after a step
    }
    guess();
  }

  while (step < target) {
    // stopping-rule state (eq. stopping): per component the minimum of the
    // earlier norms and the previous norm; per-lane norms of iterations 1, 2
    double mind[D], prv[D], dd1[D], dd2[D];
    int k = 0;
    bool ok = false, bad = false;
    for (;;) {
      ++k;
      kepler_increment<D, EXACT>(Q, hb, G, R);
      // every lane takes the 8 stages' increments
#pragma unroll
      for (int d = 0; d < D; ++d) xr[s * D + d] = R[d];
      kp_wave_sync();
#pragma unroll
      for (int j = 0; j < kS; ++j)
#pragma unroll
        for (int d = 0; d < D; ++d) Rall[d][j] = xr[j * D + d];
      kp_wave_sync();
      double qn[D], dm[D];
      if constexpr (EXACT) {
#pragma unroll
        for (int d = 0; d < D; ++d) qn[d] = stage_value<true>(T, s, qh[d], vh[d], h, Rall[d]);
      } else {
        rows_value(eta, Rall, qn);
      }
      bool nf = false, nz = false;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        dm[d] = fabs(qn[d] - Q[d]);
        nf |= !__builtin_isfinite(dm[d]);
        nz |= dm[d] != 0.0;
        Q[d] = qn[d];
      }
      bad = __ballot(nf) != 0;
      if (k <= 2) {
        // In iterations 1 and 2 the rule's minimum is still +inf, so it stops
        // only on increments that are all exactly zero; the max-norms are
        // formed only if a third iteration needs them.
        ok = __ballot(nz) == 0;
#pragma unroll
        for (int d = 0; d < D; ++d) {
          if (k == 1)
            dd1[d] = dm[d];
          else
            dd2[d] = dm[d];
        }
      } else {
        if (k == 3) {  // the rule's state after two iterations: min = norm 1, previous = norm 2
          kp_group_max(dd1);
          kp_group_max(dd2);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            mind[d] = dd1[d];
            prv[d] = dd2[d];
          }
        }
        kp_group_max(dm);
        int okl = 1;
#pragma unroll
        for (int d = 0; d < D; ++d) okl &= stop_component(dm[d], mind[d], prv[d]) ? 1 : 0;
        ok = __builtin_amdgcn_readfirstlane(okl) != 0;  // the same in every lane
      }
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
    if constexpr (EXACT) {
#pragma unroll
      for (int d = 0; d < D; ++d)
        form_update<kKepler, true>(row_tab(T), Rall[d], h, qh[d], ql[d], vh[d], vl[d]);
    } else {
      // form_update's operations (step_sums, then the two compensated
      // additions) with the nodes held in registers
      double sv[D], sc[D];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        sv[d] = Rall[d][0];
        sc[d] = cn[0] * Rall[d][0];
      }
#pragma unroll
      for (int i = 1; i < kS; ++i)
#pragma unroll
        for (int d = 0; d < D; ++d) {
          sv[d] += Rall[d][i];
          sc[d] = fma(cn[i], Rall[d][i], sc[d]);
        }
#pragma unroll
      for (int d = 0; d < D; ++d) {
        dw_add(vh[d], vl[d], sv[d]);
        dw_add(qh[d], ql[d], h * (vh[d] - sc[d]));
      }
    }
    int64_t f;
    if (frame_due(fclk, step, stride, f) && s == 0) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        a.qout[frame_index(out_off, f, D, d)] = qh[d];
        a.pout[frame_index(out_off, f, D, d)] = m * vh[d];
      }
    }
    if (step < target) guess();
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

// Batches of at most this many Kepler orbits take the latency kernel.  One
// wavefront per orbit uses 8 of its 64 lanes, but at every batch size
// measured up to this one it finished first (2,000 steps of eccentric orbits,
// against the eight-slot kernel: 128 orbits 4.0 ms against 19.9, 1,024 orbits
// 8.0 against 22.7, 8,192 orbits 14.9 against 24.9); the slots of the other
// kernel advance in lockstep at the pace of their slowest orbit.
constexpr int kKeplerLaneMaxBatch = 8192;

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

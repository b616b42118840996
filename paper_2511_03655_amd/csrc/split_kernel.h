// Persistent batched kernel for the explicit symplectic baselines of section
// 4: symmetric compositions of Strang steps (eq. Strang, eq. comp_method) run
// in their ABA form (eq. high_order_splitting) with the exact flows of eq.
// flowAB for q'' = g(q, t) (unit masses):
//
//   for j = 1..NS:  q <- q (+) fl(a_j h) v.hi;   v <- v (+) fl(b_j h) g(q.hi, t_j)
//   then            q <- q (+) fl(a_{NS+1} h) v.hi
//
// with t_j = fl(fl((n-1) h) + fl(c_j h)) (c_j: the drift fraction before the
// j-th kick) and q, v two-double values updated with the same compensated
// addition as the implicit kernels (the paper runs its splitting baselines
// with compensated summation).  One lane integrates one instance with its
// state in registers; instances come from the class queue as in the
// one-instance-per-lane implicit kernel.  Table layout:
// [a_1..a_{NS+1} | b_1..b_NS | c_1..c_NS].  The fixed-point statistics are
// zero (no iteration); a step costs NS force evaluations.
//
// Device code only: compiled at run time with hiprtc together with a user
// force (IRKGL16_USER_FORCE defined, irkgl16_user_force defined before this
// header).
#pragma once

#include "device_common.h"

namespace irk {

template <int KIND, int DQ, int NS>
__global__ __launch_bounds__(64) void split_kernel(LaunchArgs a) {
  static_assert(KIND == kUser, "split kernel: user forces only");
  const int lane = threadIdx.x;
  const ConstTab T = const_tab(a.tab);

  int inst = -1;
  bool qdone = false, taken = false;
  double h = 0.0;
  const double* prm = nullptr;
  int64_t step = 0, target = 0, stride = 1, out_off = 0, iters_off = -1, state_off = 0;
  double qh[DQ], ql[DQ], vh[DQ], vl[DQ];

  for (;;) {
    const bool fresh = take_lane_instance(a, lane, inst, qdone, taken);
    if (__ballot(inst >= 0) == 0) break;

    InstStat st0;
    if (fresh) {
      const InstDesc& dsc = a.desc[inst];
      st0 = a.stat[inst];
      h = dsc.h;
      prm = dsc.coupling_off >= 0 ? a.params + dsc.coupling_off : nullptr;
      stride = dsc.stride;
      out_off = dsc.out_off;
      iters_off = dsc.iters_off;
      state_off = dsc.state_off;
      step = st0.steps_done;
      target = launch_target(a, step, dsc.nsteps, st0.status);
      const double* St = a.state + state_off;
#pragma unroll
      for (int l = 0; l < DQ; ++l) {
        qh[l] = St[l];
        ql[l] = St[DQ + l];
        vh[l] = St[2 * DQ + l];
        vl[l] = St[3 * DQ + l];
      }
    }
    // Each lane runs its instance to the end of this launch's steps; lanes
    // of a wavefront only share the loop trip count.
    const bool live = (inst >= 0) && (step < target);
    bool bad = false;
    if (live) {
      const ConstTab r = row_tab(T);
      double ah[NS + 1], bh[NS], ch[NS];
#pragma unroll
      for (int j = 0; j <= NS; ++j) ah[j] = h * r[j];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        bh[j] = h * r[NS + 1 + j];
        ch[j] = r[2 * NS + 1 + j] * h;
      }
      while (step < target) {
        const double t_prev = (double)step * h;
        double g[DQ];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
#pragma unroll
          for (int l = 0; l < DQ; ++l) dw_add(qh[l], ql[l], ah[j] * vh[l]);
#ifdef IRKGL16_USER_FORCE
          irkgl16_user_force(qh, g, prm, t_prev + ch[j]);
#endif
#pragma unroll
          for (int l = 0; l < DQ; ++l) dw_add(vh[l], vl[l], bh[j] * g[l]);
        }
#pragma unroll
        for (int l = 0; l < DQ; ++l) dw_add(qh[l], ql[l], ah[NS] * vh[l]);
#pragma unroll
        for (int l = 0; l < DQ; ++l) bad |= !(finite(qh[l]) && finite(vh[l]));
        if (bad) break;
        if (iters_off >= 0) a.step_iters[iters_off + step] = 0;
        ++step;
        if (step % stride == 0) {
          const int64_t f = step / stride;
#pragma unroll
          for (int l = 0; l < DQ; ++l) {
            a.qout[out_off + f * DQ + l] = qh[l];
            a.pout[out_off + f * DQ + l] = vh[l];
          }
        }
      }
      if (bad) {  // non-finite: stop, remaining frames of this launch NaN
        const int64_t nfr = target / stride;
        for (int64_t f = step / stride + 1; f <= nfr; ++f) {
#pragma unroll
          for (int l = 0; l < DQ; ++l) {
            a.qout[out_off + f * DQ + l] = __builtin_nan("");
            a.pout[out_off + f * DQ + l] = __builtin_nan("");
          }
        }
      } else {
        double* St = a.state + state_off;
#pragma unroll
        for (int l = 0; l < DQ; ++l) {
          St[l] = qh[l];
          St[DQ + l] = ql[l];
          St[2 * DQ + l] = vh[l];
          St[3 * DQ + l] = vl[l];
        }
      }
      InstStat st;
      st.steps_done = step;
      st.iterations = 0;
      st.nonconv = 0;
      st.max_k = 0;
      st.status = bad ? kNonFinite : kOk;
      a.stat[inst] = st;
    }
    inst = -1;  // every taken instance is finished for this launch
  }
}

}  // namespace irk

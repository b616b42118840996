// Persistent batched IRKGL16 kernel for systems with very few position
// components (Dq <= kLaneMaxDq): one lane integrates one instance, holding all
// S x Dq stage values and increments in registers (S = 8 for IRKGL16; 2, 4
// or 6 for the lower-order members of the family).  KIND == kUserOde runs the
// first-order form instead (section 2.4, eqs. Yi2 / yn2; section 2.5, eqs.
// IRK_init / IRK_FP: y' = f(t, y), Dq = D components, stages
// Y_i = y + sum_j mu_ij L_j, update y + sum_i L_i).
//
// Each lane evaluates the force at its instance's 8 stages in turn (paper
// section 2.5: all stage evaluations of an iteration are independent), then
// performs the 8x8 stage contraction Q_i = q + h (c_i v + sum_j eta_ij R_j)
// (eq. IRK_FP2), the per-component max-norm increment and stopping rule (eqs.
// Delta_n, stopping), the compensated update (eq. qnvn2) and the extrapolated
// initial guess (eq. IRK_init2) for every component -- no LDS and no
// cross-lane traffic.  For a system of one or two bodies in the plane the
// 8-lane slot layout of the small-system kernel leaves most lanes idle in the
// contraction; here every lane of a wavefront works on its own instance.
//
// The 64 lanes of a wavefront step in lockstep: a lane whose instance has
// converged is masked until the slowest lane of the wave converges.  A lane
// whose instance finishes (or exhausts the per-launch step budget) writes the
// resumable state back and takes the next instance from the class queue (one
// atomic per wavefront for all lanes that need one).  Every lane performs its
// instance's operations in the same order as the small-system kernel, so an
// instance's results do not depend on the kernel or lane that runs it.
//
// Device code only: compiled at run time with hiprtc for a user force or
// right-hand side (the built-in Kepler increment is shared with the
// small-system kernel).
#pragma once

#include "device_common.h"

namespace irk {

constexpr int kLaneMaxDq = 4;

// R_s = h b_s g(Q_s, t_s) for the S stages of one instance.
template <int KIND, int DQ, bool EXACT, int S>
__device__ __forceinline__ void lane_increments(ConstTab T, const double (&Q)[DQ][S], double h,
                                                double G, const double* prm, int64_t step,
                                                double (&R)[DQ][S]) {
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const ConstTab r = row_tab(T);
    const double hb = h * r[Tab<S>::B + s];
    double q[DQ], out[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) q[l] = Q[l][s];
#ifdef IRKGL16_USER_FORCE
    if constexpr (KIND == kUser) user_increment<DQ>(q, hb, prm, stage_time(step, h, r[Tab<S>::C + s]), out);
#endif
#ifdef IRKGL16_USER_ODE
    if constexpr (KIND == kUserOde) ode_increment<DQ>(q, hb, prm, stage_time(step, h, r[Tab<S>::C + s]), out);
#endif
    if constexpr (KIND == kKepler) kepler_increment<DQ, EXACT>(q, hb, G, out);
#pragma unroll
    for (int l = 0; l < DQ; ++l) R[l][s] = out[l];
  }
  (void)prm;
  (void)step;
  (void)G;
}

// Schedules of the lanes of a wavefront (MODE):
//  kLaneLockstep    all live lanes iterate until the slowest converges, then
//                   all finish the step together;
//  kLaneIndependent a converged lane finishes its step in the same pass and
//                   starts the next (every pass then carries the masked
//                   end-of-step work of the lanes that finished);
//  kLaneFlush       a converged lane waits; the waiting lanes finish their
//                   steps together once half the wavefront waits, one has
//                   waited two passes, or none iterates.
// Measured on 262,144 Henon-Heiles orbits (cheap polynomial force) and
// 65,536 Schwarzschild orbits (trigonometric first-order right-hand side),
// 10^4 steps: lockstep 132.5 / 159.0 ms, flush 139.0 / 142.2 ms,
// independent 161.7 / 156.1 ms.  The default follows: lockstep for
// second-order forces, flush for first-order right-hand sides.
constexpr int kLaneLockstep = 0, kLaneIndependent = 1, kLaneFlush = 2;

template <int KIND, int DQ, bool EXACT, int S = kS,
          int MODE = (KIND == kUserOde ? kLaneFlush : kLaneLockstep)>
__global__ __launch_bounds__(64) void lane_kernel(LaunchArgs a) {
  static_assert(DQ >= 1 && DQ <= kLaneMaxDq, "lane kernel: Dq out of range");
  const int lane = threadIdx.x;
  const ConstTab T = const_tab(a.tab);

  int inst = -1;
  bool qdone = false;  // wave-uniform: the class queue is exhausted
  bool taken = false;  // single-shot launch: instances already taken
  double h = 0.0, G = 0.0;
  const double* prm = nullptr;
  int64_t step = 0, target = 0, stride = 1, out_off = 0, iters_off = -1, state_off = 0;
  int64_t it_sum = 0, nonconv = 0;
  int32_t maxk = 0;
  double qh[DQ], ql[DQ], vh[DQ], vl[DQ], mind[DQ], prv[DQ];
  double Qc[DQ][S], R[DQ][S];

  // Per step: iteration count and stopping-rule history of this lane; a
  // waiting lane's outcome (kLaneFlush).
  int k = 0;
  bool waiting = false;
  int waited = 0, kw = 0, wflags = 0;
  auto begin_step = [&]() {
    k = 0;
#pragma unroll
    for (int l = 0; l < DQ; ++l) mind[l] = prv[l] = __builtin_inf();
  };
  // One fixed-point iteration of this lane's instance: forces at the stages,
  // new stage values, increment norm and stopping rule.
  auto iterate = [&](bool& ok, bool& bad) {
    lane_increments<KIND, DQ, EXACT, S>(T, Qc, h, G, prm, step, R);
    double dmax[DQ], nf[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) dmax[l] = nf[l] = 0.0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const ConstTab r = row_tab(T);
#pragma unroll
      for (int l = 0; l < DQ; ++l) {
        const double qn = form_stage_value<KIND, EXACT>(r, s, qh[l], vh[l], h, R[l]);
        max_track(dmax[l], nf[l], fabs(qn - Qc[l][s]));
        Qc[l][s] = qn;
      }
    }
    ok = true;
    bad = false;
#pragma unroll
    for (int l = 0; l < DQ; ++l) {
      bad |= !track_finite(dmax[l], nf[l]);
      ok &= stop_component(dmax[l], mind[l], prv[l]);
    }
  };
  // End of a step after kl iterations (flags: 1 non-finite, 2 capped):
  // compensated update, output, next initial guess.  Returns whether the
  // instance is finished for this launch.
  auto end_step = [&](int kl, int flags) -> bool {
    bool rel = false;
    if (flags & 1) {  // non-finite: stop this instance, remaining frames NaN
      const int64_t nfr = target / stride;  // frames of this launch only
      for (int64_t f = step / stride + 1; f <= nfr; ++f) {
#pragma unroll
        for (int l = 0; l < DQ; ++l) {
          a.qout[out_off + f * DQ + l] = __builtin_nan("");
          if constexpr (KIND != kUserOde) a.pout[out_off + f * DQ + l] = __builtin_nan("");
        }
      }
      if (iters_off >= 0) a.step_iters[iters_off + step] = (uint8_t)kl;
      InstStat st;
      st.steps_done = step;
      st.iterations = it_sum;
      st.nonconv = nonconv;
      st.max_k = maxk;
      st.status = kNonFinite;
      a.stat[inst] = st;
      rel = true;
    } else {
      const ConstTab r = row_tab(T);
#pragma unroll
      for (int l = 0; l < DQ; ++l) form_update<KIND, EXACT>(r, R[l], h, qh[l], ql[l], vh[l], vl[l]);
      if (iters_off >= 0) a.step_iters[iters_off + step] = (uint8_t)kl;
      ++step;
      it_sum += kl;
      nonconv += (flags & 2) ? 1 : 0;
      if (kl > maxk) maxk = kl;
      if (step % stride == 0) {  // unit masses: p = v; first order: y only
        const int64_t f = step / stride;
#pragma unroll
        for (int l = 0; l < DQ; ++l) {
          a.qout[out_off + f * DQ + l] = qh[l];
          if constexpr (KIND != kUserOde) a.pout[out_off + f * DQ + l] = vh[l];
        }
      }
      if (step >= target) {
        double* St = a.state + state_off;
#pragma unroll
        for (int l = 0; l < DQ; ++l) {
          St[l] = qh[l];
          St[DQ + l] = ql[l];
          if constexpr (KIND != kUserOde) {
            St[2 * DQ + l] = vh[l];
            St[3 * DQ + l] = vl[l];
          }
#pragma unroll
          for (int s = 0; s < S; ++s) St[4 * DQ + l * S + s] = R[l][s];
        }
        InstStat st;
        st.steps_done = step;
        st.iterations = it_sum;
        st.nonconv = nonconv;
        st.max_k = maxk;
        st.status = kOk;
        a.stat[inst] = st;
        rel = true;
      } else {
        form_guess<KIND, DQ, EXACT>(T, qh, vh, R, h, Qc);
        begin_step();
      }
    }
    return rel;
  };

  for (;;) {
    // ---- lanes without an instance take the next ones from the queue
    const bool fresh = take_lane_instance(a, lane, inst, qdone, taken);
    if (__ballot(inst >= 0) == 0) break;

    if (fresh) {  // bookkeeping and state of a newly taken instance
      const InstDesc& dsc = a.desc[inst];
      const InstStat st = a.stat[inst];
      h = dsc.h;
      G = dsc.G;
      prm = dsc.coupling_off >= 0 ? a.params + dsc.coupling_off : nullptr;
      stride = dsc.stride;
      out_off = dsc.out_off;
      iters_off = dsc.iters_off;
      state_off = dsc.state_off;
      step = st.steps_done;
      it_sum = st.iterations;
      nonconv = st.nonconv;
      maxk = st.max_k;
      target = launch_target(a, step, dsc.nsteps, st.status);
      const double* St = a.state + state_off;
#pragma unroll
      for (int l = 0; l < DQ; ++l) {
        qh[l] = St[l];
        ql[l] = St[DQ + l];
        if constexpr (KIND == kUserOde) {  // first order: no velocity state
          vh[l] = vl[l] = 0.0;
        } else {
          vh[l] = St[2 * DQ + l];
          vl[l] = St[3 * DQ + l];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) R[l][s] = St[4 * DQ + l * S + s];
      }
      form_guess<KIND, DQ, EXACT>(T, qh, vh, R, h, Qc);
      begin_step();
    }

    const bool live = (inst >= 0) && (step < target);
    bool release = (inst >= 0) && !live;
    if constexpr (MODE == kLaneFlush) {
      const bool active = live && !waiting;
      if (active) {
        ++k;
        bool ok, bad;
        iterate(ok, bad);
        if (ok || bad || k >= a.max_iter) {
          waiting = true;
          waited = 0;
          kw = k;
          wflags = bad ? 1 : (!ok ? 2 : 0);
        }
      }
      const int nwait = __popcll(__ballot(waiting));
      const int nact = __popcll(__ballot(live && !waiting));
      const bool flush = nwait >= 32 || __ballot(waiting && waited >= 2) != 0 ||
                         (nwait > 0 && nact == 0);
      if (waiting) {
        if (flush) {
          waiting = false;
          release |= end_step(kw, wflags);
        } else {
          ++waited;
        }
      }
    } else if constexpr (MODE == kLaneIndependent) {
      if (live) {
        ++k;
        bool ok, bad;
        iterate(ok, bad);
        if (ok || bad || k >= a.max_iter) release |= end_step(k, bad ? 1 : (!ok ? 2 : 0));
      }
    } else {
      // One step, all live lanes in lockstep: converged lanes wait for the
      // slowest lane of the wavefront, then all finish the step together.
      bool conv = !live;
      int kl = 0, flags = 0;
      while (__ballot(!conv) != 0) {
        ++k;
        if (!conv) {
          bool ok, bad;
          iterate(ok, bad);
          if (ok || bad || k >= a.max_iter) {
            conv = true;
            kl = k;
            flags = bad ? 1 : (!ok ? 2 : 0);
          }
        }
      }
      if (live) release |= end_step(kl, flags);
    }
    if (release) inst = -1;
  }
}

}  // namespace irk

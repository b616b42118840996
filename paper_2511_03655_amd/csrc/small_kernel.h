// Persistent batched IRKGL16 kernel for small systems (Kepler, gravity with a
// handful of bodies): one 64-lane wavefront integrates 8 instances ("slots")
// at a time; a slot's 8 lanes take two roles in turn.
//
//  * stage-lane role: lane `sub` of a slot evaluates the force at stage `sub`
//    for all Dq components of its instance (paper section 2.5: the vectorised
//    f evaluates all 8 stages at once; here the 8 stages are 8 lanes);
//  * component-lane role: lane `sub` owns components sub, sub+8, sub+16 with
//    all 8 stage values in registers and performs the 8x8 stage contraction
//    Q_i = q + h (c_i v + sum_j eta_ij R_j) (eq. IRK_FP2), the per-component
//    max-norm increment and stopping rule (eqs. Delta_n, stopping), the
//    compensated update (eq. qnvn2) and the extrapolated initial guess
//    (eq. IRK_init2) without any cross-lane traffic (when Dq = 8m + 1, 2 or
//    4, the leftover components are spread over the slot by stage instead,
//    with a DPP group maximum for their increment norms).
//
// The two roles exchange stage positions and increments R_i = h b_i g(Q_i)
// through one LDS tile per slot laid out [component][stage].  Each pass of
// the wavefront is one fixed-point iteration of every slot that is still
// iterating; a slot whose instance has converged waits (its increments stay
// in its tile) and the waiting slots finish their steps together once half
// the slots wait, one has waited two passes, or none iterates -- so a slow
// instance holds the others back by at most two passes.  When an instance
// finishes, reaches the launch's step budget or limit, or (LaunchArgs.evict_k)
// has needed many iterations per step lately, its lanes write the resumable
// state back and pull the next instance from the class queue.  Each
// instance's arithmetic is independent of which slot or wave runs it, and of
// where its steps are split between launches.
//
// KIND == kUserOde runs the first-order form (section 2.4, eqs. Yi2 / yn2;
// section 2.5, eqs. IRK_init / IRK_FP) with the same two roles: stage lanes
// evaluate f(t, Y_sub), component lanes form Y_i = y + sum_j mu_ij L_j and
// update y + sum_i L_i.
//
// Device code only: the library compiles it ahead of time for the built-in
// forces (k_small.hip) and, for a user-supplied force or right-hand side, at
// run time with hiprtc (IRKGL16_USER_FORCE or IRKGL16_USER_ODE defined, the
// function defined before this header).
#pragma once

#include "device_common.h"

namespace irk {

constexpr int kSlot = 8;  // lanes per slot (one instance per slot)

// LDS tile of one slot: one row of kRow doubles per component, the stage
// values in columns 0..S-1.  The row is padded to an odd length: in the
// component-lane role the 8 lanes of a slot read rows sub, sub + 8, ... at a
// stride of kRow doubles, and an even stride would put several of them on the
// same LDS banks.  Slot tiles start 8 doubles (16 four-byte banks) apart
// modulo 16 doubles, so the two slots that one 16-lane pass of a 64-bit LDS
// access serves use disjoint banks in both roles.
template <int DQ, int S = kS>
struct SmallTile {
  static constexpr int kRow = (S % 2 == 0) ? S + 1 : S;
  static constexpr int kTile = DQ * kRow;
  static constexpr int kStride = kTile + ((8 - kTile % 16) + 16) % 16;
  static_assert(kRow % 2 == 1 && kStride % 16 == 8, "conflict-free slot tile layout");
};

// Reads the stage positions from column `sub` of the slot tile (rows of
// SmallTile::kRow doubles) and overwrites the same column with the increments
// R_sub = h b_sub g(Q_sub): a lane only touches its own column, so no barrier
// is needed between the read and the write.  Ms: the slot's masses (LDS); coef = (h b_sub) and G; prm: the
// instance's parameters of a user force; t: the stage time (user force only).
template <int KIND, int NB, int D, bool EXACT, int S = kS>
__device__ __forceinline__ void stage_increment(double* __restrict__ Xs, int sub,
                                                const double* __restrict__ Ms, double eps2,
                                                double hb, double G, const double* prm,
                                                double t) {
  constexpr int DQ = NB * D;
  constexpr int RS = SmallTile<DQ, S>::kRow;
#ifdef IRKGL16_USER_FORCE
  if constexpr (KIND == kUser) {  // R = h b_sub g(Q_sub, t_sub), g from the caller's source
    double q[DQ], r[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) q[l] = Xs[l * RS + sub];
    user_increment<DQ>(q, hb, prm, t, r);
#pragma unroll
    for (int l = 0; l < DQ; ++l) Xs[l * RS + sub] = r[l];
    return;
  }
#endif
#ifdef IRKGL16_USER_ODE
  if constexpr (KIND == kUserOde) {  // L = h b_sub f(t_sub, Y_sub), first-order form
    double y[DQ], r[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) y[l] = Xs[l * RS + sub];
    ode_increment<DQ>(y, hb, prm, t, r);
#pragma unroll
    for (int l = 0; l < DQ; ++l) Xs[l * RS + sub] = r[l];
    return;
  }
#endif
  (void)prm;
  (void)t;
  if constexpr (KIND == kKepler) {
    double q[DQ], r[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) q[l] = Xs[l * RS + sub];
    kepler_increment<DQ, EXACT>(q, hb, G, r);
#pragma unroll
    for (int l = 0; l < DQ; ++l) Xs[l * RS + sub] = r[l];
  } else if constexpr (EXACT) {
    // Ordered pairs, b ascending for every a, as in the force's definition.
    double out[DQ];
#pragma unroll
    for (int a = 0; a < NB; ++a) {
      double acc[D];
#pragma unroll
      for (int k = 0; k < D; ++k) acc[k] = 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        if (b == a) continue;
        double dx[D], r2 = 0.0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          dx[k] = Xs[(b * D + k) * RS + sub] - Xs[(a * D + k) * RS + sub];
          r2 = r2 + dx[k] * dx[k];
        }
        r2 = r2 + eps2;
        const double w = pair_weight<true>(r2, Ms[b]);
#pragma unroll
        for (int k = 0; k < D; ++k) acc[k] = acc[k] + w * dx[k];
      }
#pragma unroll
      for (int k = 0; k < D; ++k) out[a * D + k] = hb * (G * acc[k]);
    }
#pragma unroll
    for (int l = 0; l < DQ; ++l) Xs[l * RS + sub] = out[l];
  } else {
    double m[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) m[b] = Ms[b];
    double acc[DQ];
#pragma unroll
    for (int l = 0; l < DQ; ++l) acc[l] = 0.0;
    // Each unordered pair once: w = (|d|^2 + eps^2)^(-3/2) feeds both bodies.
#pragma unroll
    for (int a = 0; a < NB; ++a) {
#pragma unroll
      for (int b = a + 1; b < NB; ++b) {
        double dx[D];
#pragma unroll
        for (int k = 0; k < D; ++k) dx[k] = Xs[(b * D + k) * RS + sub] - Xs[(a * D + k) * RS + sub];
        double r2 = fma(dx[0], dx[0], eps2);
#pragma unroll
        for (int k = 1; k < D; ++k) r2 = fma(dx[k], dx[k], r2);
        const double w = rinv3(r2);
        const double wa = m[a] * w, wb = m[b] * w;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          acc[a * D + k] = fma(wb, dx[k], acc[a * D + k]);
          acc[b * D + k] = fma(-wa, dx[k], acc[b * D + k]);
        }
      }
    }
    const double coef = hb * G;
#pragma unroll
    for (int l = 0; l < DQ; ++l) Xs[l * RS + sub] = coef * acc[l];
  }
}

// Per-slot bookkeeping, kept in LDS rather than replicated in 8 lanes' VGPRs.
template <int NB>
struct SlotMeta {
  int64_t nsteps, stride, out_off, iters_off, state_off, step, target, it_sum, nonconv;
  double h, G, eps2;
  double m[NB];
  int64_t prm_off;                   // user-force parameters in the params arena, or -1
  double kema;                       // recent iterations per step (eviction, LaunchArgs.evict_k)
  int32_t inst, maxk;
};

template <int KIND, int NB, int D, bool EXACT, int S = kS>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void small_kernel(LaunchArgs a) {
  constexpr int DQ = NB * D;
  // Tail split: when Dq = 8 m + t with m >= 1 and t = 1, 2 or 4 (and one lane
  // per stage), the t components left after m full rounds are spread over
  // the slot by stage -- 8 / t lanes per tail component, t stages per lane --
  // instead of a last round in which 8 - t lanes would idle.  The lanes of a
  // tail group combine their increment norms with DPP.
  constexpr int NFULL = DQ / kSlot;
  constexpr int TAIL = DQ - NFULL * kSlot;
  constexpr bool SPLIT = (S == kSlot) && NFULL >= 1 && (TAIL == 1 || TAIL == 2 || TAIL == 4);
  constexpr int CPL = SPLIT ? NFULL : (DQ + kSlot - 1) / kSlot;  // components owned per lane
  constexpr int TG = SPLIT ? kSlot / TAIL : 1;  // lanes per tail component
  constexpr int TSL = SPLIT ? TAIL : 1;         // tail stages per lane
  constexpr int TS = SmallTile<DQ, S>::kStride;
  constexpr int RS = SmallTile<DQ, S>::kRow;
  __shared__ double X[8 * TS];
  // Coefficient table for rows picked by a lane-dependent stage (tail split).
  __shared__ double TabL[SPLIT ? Tab<S>::Size : 1];
  __shared__ SlotMeta<NB> meta[8];
  __shared__ int32_t slot_inst[8];
  __shared__ int32_t qdone;

  const int lane = threadIdx.x;
  const int slot = lane >> 3;
  const int sub = lane & 7;
  double* Xs = X + slot * TS;
  SlotMeta<NB>& M = meta[slot];
  const uint64_t smask = 0xFFull << (8 * slot);
  const ConstTab T = const_tab(a.tab);
  // Owned component cc is c = sub + 8 cc; lanes past Dq compute on a clamped
  // copy and never store.
  auto comp = [&](int cc) { return sub + kSlot * cc; };
  auto owns = [&](int cc) { return sub + kSlot * cc < DQ; };
  auto cidx = [&](int cc) { return (sub + kSlot * cc < DQ) ? sub + kSlot * cc : DQ - 1; };
  // Tail split: this lane's tail component and its first stage.
  const int tcomp = NFULL * kSlot + sub / TG;
  const int tst0 = (sub % TG) * TSL;
  const bool tlead = (sub % TG) == 0;  // writes the tail component's outputs

  int inst = -1;
  double qh[CPL] = {}, ql[CPL] = {}, vh[CPL] = {}, vl[CPL] = {}, mind[CPL] = {}, prv[CPL] = {};
  double Qc[CPL][S] = {};
  double tqh = 0.0, tql = 0.0, tvh = 0.0, tvl = 0.0, tmind = 0.0, tprv = 0.0;
  double tQ[TSL] = {};

  // Per step: iteration count, stopping-rule history, and this lane's stage
  // weight h b_sub and time t_sub (lane-dependent index: a vector load, once
  // per step).
  int k = 0;
  double hb_sub = 0.0, t_sub = 0.0;
  // A converged slot waits (its increments stay in its LDS tile) until its
  // step end runs together with other slots' (see the flush rule below):
  // kw, wok, wbad are the iteration count and outcome it converged with.
  bool waiting = false, wok = true, wbad = false;
  int waited = 0, kw = 0;
  const int sub_s = sub < S ? sub : S - 1;
  auto begin_step = [&](int64_t step) {
    k = 0;
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) mind[cc] = prv[cc] = __builtin_inf();
    tmind = tprv = __builtin_inf();
    hb_sub = M.h * T[Tab<S>::B + sub_s];
    t_sub = stage_time(step, M.h, T[Tab<S>::C + sub_s]);
  };

  if constexpr (SPLIT) {
    for (int i = lane; i < Tab<S>::Size; i += 64) TabL[i] = a.tab[i];
  }
  if (lane == 0) qdone = 0;
  if (lane < 8) {
    slot_inst[lane] = -1;
    meta[lane].inst = -1;
  }
  __syncthreads();

  for (;;) {
    if (lane < 8 && slot_inst[lane] < 0 && !qdone) {
      if (a.queue_head) {
        const int idx = atomicAdd(a.queue_head, 1);
        if (idx < queue_length(a))
          slot_inst[lane] = a.queue[idx];
        else
          qdone = 1;
      } else if (lane < a.queue_len) {
        slot_inst[lane] = a.queue[lane];  // single-shot launch: up to 8 given instances
      }
    }
    __syncthreads();
    if (!a.queue_head && lane == 0) qdone = 1;
    const int cur = slot_inst[slot];
    if (__ballot(cur >= 0) == 0) break;

    const bool fresh = cur >= 0 && cur != inst;
    if (fresh && sub == 0) {  // slot bookkeeping of a newly loaded instance
      const InstDesc& dsc = a.desc[cur];
      const InstStat st = a.stat[cur];
      M.inst = cur;
      M.h = dsc.h;
      M.G = dsc.G;
      M.eps2 = dsc.eps * dsc.eps;
      M.prm_off = dsc.coupling_off;
      M.nsteps = dsc.nsteps;
      M.stride = dsc.stride;
      M.out_off = dsc.out_off;
      M.iters_off = dsc.iters_off;
      M.state_off = dsc.state_off;
      M.step = st.steps_done;
      M.it_sum = st.iterations;
      M.nonconv = st.nonconv;
      M.maxk = st.max_k;
      M.target = launch_target(a, st.steps_done, dsc.nsteps, st.status);
      M.kema = 2.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) M.m[b] = (dsc.mass_off >= 0) ? a.params[dsc.mass_off + b] : 1.0;
    }
    __syncthreads();
    if (fresh) inst = cur;
    if (fresh && M.step < M.target) {  // component state of the new instance
      const double* St = a.state + M.state_off;
      double Rp[CPL][S];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        const int c = cidx(cc);
        qh[cc] = St[c];
        ql[cc] = St[DQ + c];
        vh[cc] = St[2 * DQ + c];
        vl[cc] = St[3 * DQ + c];
#pragma unroll
        for (int s = 0; s < S; ++s) Rp[cc][s] = St[4 * DQ + c * S + s];
      }
      form_guess<KIND, CPL, EXACT>(T, qh, vh, Rp, M.h, Qc);
      if constexpr (SPLIT) {
        tqh = St[tcomp];
        tql = St[DQ + tcomp];
        tvh = St[2 * DQ + tcomp];
        tvl = St[3 * DQ + tcomp];
        double tRp[S];
#pragma unroll
        for (int s = 0; s < S; ++s) tRp[s] = St[4 * DQ + tcomp * S + s];
#pragma unroll
        for (int u = 0; u < TSL; ++u)
          tQ[u] = guess_stage<KIND, EXACT>(TabL, tst0 + u, tqh, tvh, tRp, M.h);
      }
    }

    // ---- one fixed-point iteration for every live slot.  A slot whose
    // instance has converged finishes its step in the same pass and starts
    // the next one, so no slot waits for a slower one (a slow instance costs
    // only its own slot's throughput).
    const bool live = (inst >= 0) && (M.step < M.target);
    const double h = M.h;
    if (fresh) {
      begin_step(M.step);
      waiting = false;
    }
    const bool active = live && !waiting;  // iterates in this pass
    if (active) {
      ++k;
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        if (owns(cc)) {
#pragma unroll
          for (int s = 0; s < S; ++s) Xs[comp(cc) * RS + s] = Qc[cc][s];
        }
      }
      if constexpr (SPLIT) {
#pragma unroll
        for (int u = 0; u < TSL; ++u) Xs[tcomp * RS + tst0 + u] = tQ[u];
      }
    }
    __syncthreads();
    if (active && sub < S)  // lanes past the stage count idle in this role
      stage_increment<KIND, NB, D, EXACT, S>(Xs, sub, M.m, M.eps2, hb_sub, M.G,
                                             M.prm_off >= 0 ? a.params + M.prm_off : nullptr,
                                             t_sub);
    __syncthreads();
    bool ok = true, bad = false;
    if (active) {
      double R[CPL][S], dmax[CPL], nf[CPL];
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        dmax[cc] = 0.0;
        nf[cc] = 0.0;
#pragma unroll
        for (int s = 0; s < S; ++s) R[cc][s] = Xs[cidx(cc) * RS + s];
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const ConstTab r = row_tab(T);
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
          const double qn = form_stage_value<KIND, EXACT>(r, s, qh[cc], vh[cc], h, R[cc]);
          max_track(dmax[cc], nf[cc], fabs(qn - Qc[cc][s]));
          Qc[cc][s] = qn;
        }
      }
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc) {
        if (owns(cc)) {
          bad |= !track_finite(dmax[cc], nf[cc]);
          ok &= stop_component(dmax[cc], mind[cc], prv[cc]);
        }
      }
      if constexpr (SPLIT) {  // this lane's stages of its tail component
        double tR[S];
#pragma unroll
        for (int s = 0; s < S; ++s) tR[s] = Xs[tcomp * RS + s];
        double tdmax = 0.0, tnf = 0.0;
#pragma unroll
        for (int u = 0; u < TSL; ++u) {
          const double qn = form_stage_value<KIND, EXACT>(TabL, tst0 + u, tqh, tvh, h, tR);
          max_track(tdmax, tnf, fabs(qn - tQ[u]));
          tQ[u] = qn;
        }
        group_track<TG>(tdmax, tnf);
        bad |= !track_finite(tdmax, tnf);
        ok &= stop_component(tdmax, tmind, tprv);
      }
    }
    const uint64_t okm = __ballot(ok);
    const uint64_t badm = __ballot(bad);
    const bool slot_ok = (okm & smask) == smask;
    const bool slot_bad = (badm & smask) != 0;
    if (active && (slot_ok || slot_bad || k >= a.max_iter)) {
      waiting = true;
      waited = 0;
      kw = k;
      wok = slot_ok;
      wbad = slot_bad;
    }
    // Flush rule: the waiting slots finish their steps together once at
    // least half the slots wait, once one has waited two passes, or once no
    // slot is iterating.  The step end then runs about once per step for the
    // whole wavefront instead of in nearly every pass, while a slot that
    // needs many iterations never holds the others back for long.
    const int nwait = __popcll(__ballot(waiting && sub == 0));
    const int nact = __popcll(__ballot(live && !waiting && sub == 0));
    const bool flush =
        nwait >= kSlot / 2 || __ballot(waiting && waited >= 2) != 0 || (nwait > 0 && nact == 0);
    const bool done = waiting && flush;
    if (waiting && !flush) ++waited;
    // A wavefront holding an instance deep in its fixed-point iteration
    // (k >= 4 this step; typical steps take 2 or 3) takes issue priority on
    // its SIMD: the long sequential integrations, which bound the batch's
    // completion time, then run near their uncontended speed while the
    // other wavefronts fill the remaining issue slots.
    if (__ballot(active && k >= 4) != 0)
      __builtin_amdgcn_s_setprio(2);
    else
      __builtin_amdgcn_s_setprio(0);

    // ---- end of the step for the slots that converged: compensated update,
    // output, next initial guess
    bool release = (inst >= 0) && !live;
    if (done) {
      waiting = false;
      const int kslot = kw;
      const int64_t step0 = M.step, stride = M.stride, out_off = M.out_off;
      if (wbad) {  // non-finite: stop this instance, remaining frames NaN
        const int64_t nf = last_frame_of_launch(M.target, stride);  // frames of this launch only
        for (int64_t f = first_nan_frame(step0, stride); f <= nf; ++f) {
#pragma unroll
          for (int cc = 0; cc < CPL; ++cc) {
            if (owns(cc)) {
              a.qout[frame_index(out_off, f, DQ, comp(cc))] = __builtin_nan("");
              if constexpr (KIND != kUserOde)
                a.pout[frame_index(out_off, f, DQ, comp(cc))] = __builtin_nan("");
            }
          }
          if (SPLIT && tlead) {
            a.qout[frame_index(out_off, f, DQ, tcomp)] = __builtin_nan("");
            if constexpr (KIND != kUserOde) a.pout[frame_index(out_off, f, DQ, tcomp)] = __builtin_nan("");
          }
        }
        if (sub == 0) {
          if (M.iters_off >= 0) a.step_iters[iters_index(M.iters_off, step0)] = (uint8_t)kslot;
          InstStat st;
          st.steps_done = step0;
          st.iterations = M.it_sum;
          st.nonconv = M.nonconv;
          st.max_k = M.maxk;
          st.status = kNonFinite;
          a.stat[inst] = st;
        }
        release = true;
      } else {
        const int64_t step = step0 + 1;
        const bool frame = (step % stride) == 0;
        const bool last = step >= M.target;
        // An instance whose recent steps needed many iterations stops here,
        // for the next launch to move it to the stage-parallel kernel.
        const double kema = 0.875 * M.kema + 0.125 * (double)kslot;
        const bool evict = !last && a.evict_k > 0.0 && kema >= a.evict_k;
        const bool stop = last || evict;
        double R[CPL][S];
        const ConstTab r = row_tab(T);
#pragma unroll
        for (int cc = 0; cc < CPL; ++cc) {
#pragma unroll
          for (int s = 0; s < S; ++s) R[cc][s] = Xs[cidx(cc) * RS + s];
          form_update<KIND, EXACT>(r, R[cc], h, qh[cc], ql[cc], vh[cc], vl[cc]);
          if (owns(cc)) {
            const int c = comp(cc);
            if (frame) {
              const int64_t f = step / stride;
              a.qout[frame_index(out_off, f, DQ, c)] = qh[cc];
              if constexpr (KIND != kUserOde)
                a.pout[frame_index(out_off, f, DQ, c)] = M.m[c / D] * vh[cc];
            }
            if (stop) {
              a.state[state_index(M.state_off, DQ, 0, c)] = qh[cc];
              a.state[state_index(M.state_off, DQ, 1, c)] = ql[cc];
              a.state[state_index(M.state_off, DQ, 2, c)] = vh[cc];
              a.state[state_index(M.state_off, DQ, 3, c)] = vl[cc];
#pragma unroll
              for (int s = 0; s < S; ++s) a.state[rprev_index(M.state_off, DQ, c, s, S)] = R[cc][s];
            }
          }
        }
        if (!stop) {
          form_guess<KIND, CPL, EXACT>(T, qh, vh, R, h, Qc);
          begin_step(step);
        }
        if constexpr (SPLIT) {  // tail component: update (replicated), outputs, guess
          double tR[S];
#pragma unroll
          for (int s = 0; s < S; ++s) tR[s] = Xs[tcomp * RS + s];
          form_update<KIND, EXACT>(r, tR, h, tqh, tql, tvh, tvl);
          if (tlead) {
            if (frame) {
              const int64_t f = step / stride;
              a.qout[frame_index(out_off, f, DQ, tcomp)] = tqh;
              if constexpr (KIND != kUserOde)
                a.pout[frame_index(out_off, f, DQ, tcomp)] = M.m[tcomp / D] * tvh;
            }
            if (stop) {
              a.state[state_index(M.state_off, DQ, 0, tcomp)] = tqh;
              a.state[state_index(M.state_off, DQ, 1, tcomp)] = tql;
              a.state[state_index(M.state_off, DQ, 2, tcomp)] = tvh;
              a.state[state_index(M.state_off, DQ, 3, tcomp)] = tvl;
#pragma unroll
              for (int s = 0; s < S; ++s) a.state[rprev_index(M.state_off, DQ, tcomp, s, S)] = tR[s];
            }
          }
          if (!stop) {
#pragma unroll
            for (int u = 0; u < TSL; ++u)
              tQ[u] = guess_stage<KIND, EXACT>(TabL, tst0 + u, tqh, tvh, tR, h);
          }
        }
        if (sub == 0) {
          if (M.iters_off >= 0) a.step_iters[iters_index(M.iters_off, step0)] = (uint8_t)kslot;
          M.step = step;
          M.it_sum += kslot;
          M.nonconv += wok ? 0 : 1;
          M.kema = kema;
          if (kslot > M.maxk) M.maxk = kslot;
          if (evict) a.evicted[inst] = 1;
          if (stop) {
            InstStat st;
            st.steps_done = step;
            st.iterations = M.it_sum;
            st.nonconv = M.nonconv;
            st.max_k = M.maxk;
            st.status = kOk;
            a.stat[inst] = st;
          }
        }
        release = stop;
      }
    }
    __syncthreads();
    if (release) {
      if (sub == 0) slot_inst[slot] = -1;
      inst = -1;
    }
    __syncthreads();
  }
}

}  // namespace irk

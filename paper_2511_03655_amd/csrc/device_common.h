// Device-side building blocks shared by the IRKGL16 kernels (gfx950, FP64).
//
// Everything here is compiled with -ffp-contract=off: a product is only fused
// into an fma where the code says fma(), so the two-double state updates keep
// their exact error terms.
#pragma once

#ifndef __HIPCC_RTC__  // run-time compilation provides these itself
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "irkgl16_coeffs.h"

namespace irk {

#ifdef __HIPCC_RTC__  // fixed-width integer names without the C headers
typedef long long int64_t;
typedef int int32_t;
typedef unsigned int uint32_t;
typedef unsigned long long uint64_t;
typedef unsigned char uint8_t;
#endif

}  // namespace irk

#include "store_index.h"

namespace irk {

constexpr int kS = 8;  // stages

// Force kinds (same numbering as the C ABI).
constexpr int kKepler = 0;
constexpr int kGravity = 1;
constexpr int kChain = 2;
constexpr int kUser = 3;     // force g(q, t) given as device source, compiled at run time
constexpr int kUserOde = 4;  // first-order right-hand side f(t, y) given as device source

// Per-instance status codes (same numbering as the C ABI).
constexpr int kOk = 0;
constexpr int kNonFinite = -4;

// Device descriptor of one instance.  Offsets are in doubles (or bytes for
// step_iters) into the context's arenas.
struct InstDesc {
  int64_t state_off;  // [q_hi, q_lo, v_hi, v_lo] x Dq, then R_prev as [Dq][8]
  int64_t in_off;     // q0/p0 offset
  int64_t out_off;    // first frame in q_out/p_out ([frame][Dq])
  int64_t iters_off;  // per-step iteration counts, or -1
  int64_t nsteps;
  int64_t stride;
  double h, G, eps, beta;
  int64_t mass_off;      // n masses (GRAVITY, CHAIN) or -1 (all ones)
  int64_t coupling_off;  // n+1 stiffnesses (CHAIN) or -1 (all ones)
  int32_t kind, n, d, pad;
};

// Per-instance results, persistent across launches (resumable state).
struct InstStat {
  int64_t steps_done;
  int64_t iterations;
  int64_t nonconv;
  int32_t max_k;
  int32_t status;
};

// Coefficient table in device memory, read with wave-uniform (scalar) loads so
// that the 8x8 tables live in SGPRs/scalar cache rather than as materialised
// 64-bit immediates in vector registers.  Layout (doubles):
// [0,8) c, [8,16) b, [16,80) eta, [80,144) mu, [144,208) nu, [208,272) K
// (row-major, row = stage formed, column = stage summed over).
constexpr int kTabC = 0, kTabB = 8, kTabEta = 16, kTabMu = 80, kTabNu = 144, kTabK = 208,
              kTabSize = 272;

// The same layout for the s-stage member of the family (s = 2, 4, 6, 8):
// [c | b | eta | mu | nu | K], s x s matrices row-major.  Tab<8> is the table
// above.
template <int S>
struct Tab {
  static constexpr int C = 0, B = S, Eta = 2 * S, Mu = 2 * S + S * S, Nu = 2 * S + 2 * S * S,
                       K = 2 * S + 3 * S * S, Size = 2 * S + 4 * S * S;
};
static_assert(Tab<8>::K == kTabK && Tab<8>::Size == kTabSize, "table layout");

// Pointer into the constant address space: loads through it with uniform
// indices become scalar (SMEM) loads.
typedef const __attribute__((address_space(4))) double* ConstTab;

__device__ __forceinline__ ConstTab const_tab(const double* p) { return (ConstTab)p; }

// Returns the same pointer, but opaque to the optimiser: loads through the
// result cannot be hoisted above this point.  Used once per coefficient row so
// that only the row in use occupies scalar registers (hoisting all 208
// coefficients out of the step loop overflows the SGPR file).
__device__ __forceinline__ ConstTab row_tab(ConstTab p) {
  asm volatile("" : "+s"(p));
  return p;
}

// Wavefronts per CU that one batched class's persistent grid may occupy (the
// classes of a call run concurrently; a class that filled every CU with its
// own workgroups would lock the others out of LDS and wave slots).
constexpr int kClassWavesPerCu = 8;

// Workgroups per CU for a persistent grid of `waves_per_wg`-wave workgroups:
// at most what the occupancy calculator allows and within the class budget.
inline int class_blocks_per_cu(int occupancy_per_cu, int waves_per_wg) {
  int b = kClassWavesPerCu / (waves_per_wg > 0 ? waves_per_wg : 1);
  if (b < 1) b = 1;
  return b < occupancy_per_cu ? b : occupancy_per_cu;
}

// Stage time t_{n-1} + c_i h of eq. IRK_FP for a step that starts after
// `steps` steps from t = 0, rounded as fl(fl(steps h) + fl(c_i h)) (all HIP
// code is compiled without contraction).
__device__ __forceinline__ double stage_time(int64_t steps, double h, double c) {
  const double t_prev = (double)steps * h;
  const double ch = c * h;
  return t_prev + ch;
}

struct LaunchArgs {
  const double* tab;
  const InstDesc* desc;
  InstStat* stat;
  double* state;
  const double* params;
  double* qout;
  double* pout;
  uint8_t* step_iters;
  const int32_t* queue;  // instance ids of this class, in processing order
  int32_t queue_len;
  int32_t max_iter;
  int32_t* queue_head;   // atomic work counter (zeroed by the prepare kernel)
  int64_t step_budget;   // max steps per instance in this launch (<= 0: all)
  int32_t exact;         // reproducible arithmetic (see the EXACT policies below)
  // If set, the queue length in device memory (written by an earlier kernel
  // of the same call); replaces queue_len for launches with a queue counter.
  const int32_t* queue_len_dev = nullptr;
  // If > 0: no instance goes past this step count in this launch (a chunk
  // boundary; instances behind it catch up).
  int64_t step_limit = 0;
  // Small-system kernel, if > 0: an instance whose recent iterations per step
  // (an exponential average over about 8 steps) reach evict_k stops at the
  // end of that step, with `evicted` set, for the next launch to move it to
  // the stage-parallel kernel.
  double evict_k = 0.0;
  uint8_t* evicted = nullptr;
  // Stage-parallel kernel: the launch serves promoted instances, the slowest
  // work of the call, whose wavefronts then take the highest issue priority.
  int32_t promoted = 0;
};

// Step count an instance may reach in a launch: its own, cut by the launch's
// step budget (relative) and step limit (absolute); its current count if it
// has stopped or is already past the limit.
__device__ __forceinline__ int64_t launch_target(const LaunchArgs& a, int64_t steps_done,
                                                 int64_t nsteps, int32_t status) {
  return launch_target_of(steps_done, nsteps, status == kOk, a.step_budget, a.step_limit);
}

// Length of a launch's class queue.
__device__ __forceinline__ int32_t queue_length(const LaunchArgs& a) {
  return a.queue_len_dev ? *a.queue_len_dev : a.queue_len;
}

// One-instance-per-lane kernels: lanes without an instance (inst < 0) take the
// next ones from the class queue, one atomic per wavefront for all of them
// (single-shot launches without a queue counter take up to 64 given
// instances once).  qdone (wave-uniform) marks an exhausted queue.  Returns
// true for a lane that took a new instance.
__device__ __forceinline__ bool take_lane_instance(const LaunchArgs& a, int lane, int& inst,
                                                   bool& qdone, bool& taken) {
  bool fresh = false;
  if (a.queue_head) {
    if (!qdone) {
      const uint64_t need = __ballot(inst < 0);
      if (need != 0) {
        const int cnt = __popcll(need);
        const int leader = __ffsll((unsigned long long)need) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(a.queue_head, cnt);
        base = __shfl(base, leader, 64);
        if (inst < 0) {
          const int idx = base + __popcll(need & ((1ull << lane) - 1ull));
          if (idx < queue_length(a)) {
            inst = a.queue[idx];
            fresh = true;
          }
        }
        if (base + cnt >= queue_length(a)) qdone = true;
      }
    }
  } else if (!taken) {
    taken = true;
    if (lane < a.queue_len) {
      inst = a.queue[lane];
      fresh = true;
    }
  }
  return fresh;
}

// x (+) d on a two-double value: (s, e) = TwoSum(hi, d); t = e + lo;
// (hi, lo) = Fast2Sum(s, t).
__device__ __forceinline__ void dw_add(double& hi, double& lo, double d) {
  const double s = hi + d;
  const double bv = s - hi;
  const double e = (hi - (s - bv)) + (d - bv);
  const double t = e + lo;
  const double h2 = s + t;
  lo = t - (h2 - s);
  hi = h2;
}

// r2^(-3/2) for r2 > 0: the hardware reciprocal square root (about 24
// correct bits) refined by two Newton-Raphson steps y <- y + y (1/2 - (r2/2) y^2)
// (result within 1 ulp of r2^(-1/2)), then cubed.
__device__ __forceinline__ double rinv3(double r2) {
  const double hr = 0.5 * r2;
  double y = __builtin_amdgcn_rsq(r2);
  double t = hr * y;
  double e = fma(-t, y, 0.5);
  y = fma(y, e, y);
  t = hr * y;
  e = fma(-t, y, 0.5);
  y = fma(y, e, y);
  return (y * y) * y;
}

// Stopping rule of eq. stopping for one component: `mind` = min(Delta[1..k-2]),
// `prev` = Delta[k-1], both +inf before the first iteration.  Returns whether
// this component allows stopping and advances the history.
__device__ __forceinline__ bool stop_component(double delta, double& mind, double& prev) {
  const double m = (prev < delta) ? prev : delta;
  const bool ok = (delta == 0.0) || (mind <= m);
  if (prev < mind) mind = prev;
  prev = delta;
  return ok;
}

__device__ __forceinline__ bool finite(double x) { return x - x == 0.0; }

// NaN-keeping running maximum of |differences|.
__device__ __forceinline__ double max_keep_nan(double acc, double a) {
  return (a != a || a > acc) ? a : acc;
}

// Running maximum of non-negative increments with non-finite tracking: fmax
// (one instruction) drops a NaN operand, so non-finite increments are recorded
// in `nf` instead (d * 0 is NaN exactly when d is not finite; otherwise nf
// stays +0).  The maximum of finite increments is exact, as with
// max_keep_nan.
__device__ __forceinline__ void max_track(double& acc, double& nf, double d) {
  acc = fmax(acc, d);
  nf = fma(d, 0.0, nf);
}

// True when the tracked maximum is finite and no non-finite increment occurred.
__device__ __forceinline__ bool track_finite(double acc, double nf) {
  return finite(acc) && nf == 0.0;
}

// A double taken from another lane of the wavefront by a DPP pattern (CTRL:
// 0xB1 = lane xor 1 and 0x4E = lane xor 2 within a quad, 0x141 = mirror
// within each 8-lane half row).  Every lane of the group must be active.
template <int CTRL>
__device__ __forceinline__ double dpp_double(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Combines a tracked maximum (max_track) over aligned groups of G = 2, 4 or 8
// lanes: the maximum is exact in any order and a non-finite mark anywhere
// reaches every lane of the group.
template <int G>
__device__ __forceinline__ void group_track(double& acc, double& nf) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8, "group of 1, 2, 4 or 8 lanes");
  if constexpr (G >= 2) {
    acc = fmax(acc, dpp_double<0xB1>(acc));
    nf = nf + dpp_double<0xB1>(nf);
  }
  if constexpr (G >= 4) {
    acc = fmax(acc, dpp_double<0x4E>(acc));
    nf = nf + dpp_double<0x4E>(nf);
  }
  if constexpr (G >= 8) {  // quads are uniform now: the mirror pairs quad 0 with quad 1
    acc = fmax(acc, dpp_double<0x141>(acc));
    nf = nf + dpp_double<0x141>(nf);
  }
}


// ---------------------------------------------------------------------------
// Arithmetic policies.  EXACT = false: fused multiply-adds and the refined
// reciprocal square root (fastest).  EXACT = true: the reference operation
// order of a plain IEEE implementation -- separate multiply and add, sums from
// 0.0 in ascending index order, correctly rounded sqrt and division -- so that
// results are bit-identical to a strict-IEEE CPU evaluation of the same
// formulas.

// The helpers below are generic in the stage count S (deduced from the
// length of the stage arrays; 8 for IRKGL16) and read the table of Tab<S>.

// sum_j w[off + j] x[j], j = 0..S-1
template <bool EXACT, int S, class W>
__device__ __forceinline__ double row_dot(W w, int off, const double (&x)[S]) {
  if constexpr (EXACT) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < S; ++j) s = s + w[off + j] * x[j];
    return s;
  } else {
    double s = w[off] * x[0];
#pragma unroll
    for (int j = 1; j < S; ++j) s = fma(w[off + j], x[j], s);
    return s;
  }
}

// Stage value q + h (c_s v + sum_j M_sj R_j) with M = eta (eqs. Qi2 /
// IRK_FP2), or M = K for the folded initial guess.
template <bool EXACT, int S, class W>
__device__ __forceinline__ double stage_value(W w, int s, double q, double v, double h,
                                              const double (&R)[S], int mat = Tab<S>::Eta) {
  if constexpr (EXACT) {
    return q + h * (w[Tab<S>::C + s] * v + row_dot<true>(w, mat + s * S, R));
  } else {
    double acc = w[Tab<S>::C + s] * v;
#pragma unroll
    for (int j = 0; j < S; ++j) acc = fma(w[mat + s * S + j], R[j], acc);
    return fma(h, acc, q);
  }
}

// sum_i R_i and sum_i c_i R_i (eq. qnvn2).
template <bool EXACT, int S>
__device__ __forceinline__ void step_sums(ConstTab w, const double (&R)[S], double& sv,
                                          double& sc) {
  if constexpr (EXACT) {
    sv = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) sv = sv + R[i];
    sc = row_dot<true>(w, Tab<S>::C, R);
  } else {
    sv = R[0];
#pragma unroll
    for (int i = 1; i < S; ++i) sv += R[i];
    sc = row_dot<false>(w, Tab<S>::C, R);
  }
}

// (|d|^2 + eps^2)^(-3/2) times m: fast form via the refined reciprocal square
// root, exact form m / (r2 sqrt(r2)) with correctly rounded sqrt and division.
template <bool EXACT>
__device__ __forceinline__ double pair_weight(double r2, double m) {
  if constexpr (EXACT) {
    return m / (r2 * sqrt(r2));
  } else {
    return m * rinv3(r2);
  }
}

// Stage increment R = h b_s g(q) of the Kepler force g = -G q / |q|^3 for one
// stage value q.
template <int DQ, bool EXACT>
__device__ __forceinline__ void kepler_increment(const double (&q)[DQ], double hb, double G,
                                                 double (&R)[DQ]) {
  if constexpr (EXACT) {  // g = -G q / (r2 sqrt(r2))
    double r2 = 0.0;
#pragma unroll
    for (int l = 0; l < DQ; ++l) r2 = r2 + q[l] * q[l];
    const double r3 = r2 * sqrt(r2);
#pragma unroll
    for (int l = 0; l < DQ; ++l) R[l] = hb * (-G * q[l] / r3);
  } else {
    double r2 = q[0] * q[0];
#pragma unroll
    for (int l = 1; l < DQ; ++l) r2 = fma(q[l], q[l], r2);
    const double w = -(hb * G) * rinv3(r2);
#pragma unroll
    for (int l = 0; l < DQ; ++l) R[l] = w * q[l];
  }
}

#ifdef IRKGL16_USER_FORCE
// Stage increment R = h b_s g(q, t) of a force supplied as source (defined
// before this header in the run-time compiled program).
template <int DQ>
__device__ __forceinline__ void user_increment(const double (&q)[DQ], double hb, const double* prm,
                                               double t, double (&R)[DQ]) {
  double g[DQ];
  irkgl16_user_force(q, g, prm, t);
#pragma unroll
  for (int l = 0; l < DQ; ++l) R[l] = hb * g[l];
}
#endif

// Initial guess for the owned components from their previous-step increments
// Rp (eq. IRK_init2): V0_i = v + sum_j nu_ij Rp_j, L0_j = h b_j V0_j,
// Q_i = q + sum_j mu_ij L0_j, in that order with EXACT.  The fused mode
// evaluates the same linear map folded into one matrix,
// Q_i = q + h (c_i v + sum_j K_ij Rp_j) with K = A W diag(1/b) (80 instead of
// 144 operations per component).  Rows are fetched one at a time.
template <int CPL, bool EXACT, int S>
__device__ __forceinline__ void initial_guess(ConstTab T, const double (&qh)[CPL],
                                              const double (&vh)[CPL], const double (&Rp)[CPL][S],
                                              double h, double (&Q)[CPL][S]) {
  if constexpr (!EXACT) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const ConstTab r = row_tab(T);
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc)
        Q[cc][s] = stage_value<false>(r, s, qh[cc], vh[cc], h, Rp[cc], Tab<S>::K);
    }
    return;
  }
  double L0[CPL][S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const ConstTab r = row_tab(T);
    const double hb = h * r[Tab<S>::B + s];
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc)
      L0[cc][s] = hb * (vh[cc] + row_dot<EXACT>(r, Tab<S>::Nu + s * S, Rp[cc]));
  }
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const ConstTab r = row_tab(T);
#pragma unroll
    for (int cc = 0; cc < CPL; ++cc) Q[cc][s] = qh[cc] + row_dot<EXACT>(r, Tab<S>::Mu + s * S, L0[cc]);
  }
}

// ---- first-order (mu) form, eqs. Yi2 / yn2, IRK_init / IRK_FP
// Stage value Y_s = y + sum_j M_sj L_j with M = mu (iteration) or nu (initial
// guess from the previous step's increments).
template <bool EXACT, int S, class W>
__device__ __forceinline__ double ode_stage_value(W w, int s, double y, const double (&L)[S],
                                                  int mat) {
  return y + row_dot<EXACT>(w, mat + s * S, L);
}

// sum_i L_i (eq. yn2).
template <bool EXACT, int S>
__device__ __forceinline__ double ode_step_sum(const double (&L)[S]) {
  if constexpr (EXACT) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < S; ++i) s = s + L[i];
    return s;
  } else {
    double s = L[0];
#pragma unroll
    for (int i = 1; i < S; ++i) s += L[i];
    return s;
  }
}

#ifdef IRKGL16_USER_ODE
// Stage increment L = h b_s f(t, y) of a right-hand side supplied as source.
template <int DQ>
__device__ __forceinline__ void ode_increment(const double (&y)[DQ], double hb, const double* prm,
                                              double t, double (&L)[DQ]) {
  double f[DQ];
  irkgl16_user_rhs(y, f, prm, t);
#pragma unroll
  for (int l = 0; l < DQ; ++l) L[l] = hb * f[l];
}
#endif

// ---- the two forms behind one interface (KIND == kUserOde: first order)
// Initial guess for CPL owned components from the previous step's increments.
template <int KIND, int CPL, bool EXACT, int S>
__device__ __forceinline__ void form_guess(ConstTab T, const double (&qh)[CPL],
                                           const double (&vh)[CPL], const double (&Rp)[CPL][S],
                                           double h, double (&Q)[CPL][S]) {
  if constexpr (KIND == kUserOde) {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const ConstTab r = row_tab(T);
#pragma unroll
      for (int cc = 0; cc < CPL; ++cc)
        Q[cc][s] = ode_stage_value<EXACT>(r, s, qh[cc], Rp[cc], Tab<S>::Nu);
    }
  } else {
    initial_guess<CPL, EXACT>(T, qh, vh, Rp, h, Q);
  }
}

// Initial guess of one stage s of one component: the same operations, in the
// same order, as form_guess for that stage (the table may be indexed with a
// lane-dependent s).
template <int KIND, bool EXACT, int S, class W>
__device__ __forceinline__ double guess_stage(W T, int s, double q, double v,
                                              const double (&Rp)[S], double h) {
  if constexpr (KIND == kUserOde) {
    return ode_stage_value<EXACT>(T, s, q, Rp, Tab<S>::Nu);
  } else if constexpr (!EXACT) {
    return stage_value<false>(T, s, q, v, h, Rp, Tab<S>::K);
  } else {
    double L0[S];
#pragma unroll
    for (int j = 0; j < S; ++j)
      L0[j] = (h * T[Tab<S>::B + j]) * (v + row_dot<true>(T, Tab<S>::Nu + j * S, Rp));
    return q + row_dot<true>(T, Tab<S>::Mu + s * S, L0);
  }
}

// New stage value of one component from the current increments.
template <int KIND, bool EXACT, int S, class W>
__device__ __forceinline__ double form_stage_value(W r, int s, double q, double v, double h,
                                                   const double (&R)[S]) {
  if constexpr (KIND == kUserOde) {
    return ode_stage_value<EXACT>(r, s, q, R, Tab<S>::Mu);
  } else {
    return stage_value<EXACT>(r, s, q, v, h, R);
  }
}

// Compensated end-of-step update of one component (eq. yn2 or eq. qnvn2).
template <int KIND, bool EXACT, int S>
__device__ __forceinline__ void form_update(ConstTab r, const double (&R)[S], double h, double& qh,
                                            double& ql, double& vh, double& vl) {
  if constexpr (KIND == kUserOde) {
    dw_add(qh, ql, ode_step_sum<EXACT>(R));
  } else {
    double sv, sc;
    step_sums<EXACT>(r, R, sv, sc);
    dw_add(vh, vl, sv);
    dw_add(qh, ql, h * (vh - sc));
  }
}


}  // namespace irk

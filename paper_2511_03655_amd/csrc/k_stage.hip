// Persistent stage-parallel IRKGL16 kernel for gravitational systems of up to
// 128 bodies (few-body and medium systems: 16- and 64-body planetary systems,
// small clusters), in d = 1, 2 or 3 dimensions.
//
// Mapping: one workgroup integrates one system at a time; lane (u, s) with
// lane id 8 u + s owns body u at stage s.  A system of n bodies uses
// 8 np lanes, np = n rounded up to a multiple of 8, so the 8 stage lanes of a
// body always sit in one wavefront.  Per fixed-point iteration:
//  * force: lane (u, s) sums m_b (Q_b,s - Q_u,s) r^-3 over the sources b in
//    ascending order, reading the stage-s positions of the sources from an LDS
//    tile [b][s][xyz] (8 distinct addresses per wavefront read, one per stage,
//    each broadcast to 8 lanes), and forms R_s = h b_s G g_s (eq. IRK_FP2);
//  * stage update: the body's 8 increments R_j are exchanged through LDS inside
//    the wavefront (no workgroup barrier), and lane (u, s) forms its new stage
//    value Q_s = q + h (c_s v + sum_j eta_sj R_j) with the row eta_s held in
//    registers;
//  * convergence: the per-component max-norm increment over the 8 stages
//    (eq. Delta_n) is a butterfly reduction over the 8 stage lanes; the stopping
//    rule (eq. stopping) runs redundantly in those lanes, and a workgroup flag
//    collects "not yet converged" over all components.
// The stage positions are double-buffered in LDS, so one workgroup barrier per
// iteration suffices.  After convergence the compensated update (eq. qnvn2) is
// done redundantly by the 8 stage lanes of each body (stage-0 lanes write
// outputs and state), and each lane forms its own stage of the next initial
// guess (eq. IRK_init2).
#include "device_common.h"

namespace irk {

constexpr int kStageMaxBodies = 128;

// Component stride of a body's stage position in the LDS tiles: odd (D, or
// D + 1 for even D), so that the 8 stage addresses of one source in the force
// loop, the per-lane writes of R and Q, and the two bodies' broadcast reads of
// R that one 16-lane pass of a 64-bit LDS access serves all fall on distinct
// four-byte banks.
template <int D>
constexpr int stage_pad() {
  static_assert(D >= 1 && D <= 3, "d = 1, 2 or 3");
  return (D % 2 == 1) ? D : D + 1;
}

// LDS doubles: Qt [2][np][8][P], Rt [np][8][P], masses [np]; then 8 int32.
template <int D>
size_t stage_lds_doubles(int np) {
  constexpr int P = stage_pad<D>();
  return (size_t)3 * np * kS * P + np;
}

// Maximum over the 8 stage lanes of a body (lanes 8u .. 8u+7, all active or
// all inactive together) by DPP: swap neighbours, swap pairs, then mirror
// within the 8 lanes, which pairs each quad with the other.  The maximum is
// exact in any order.  A non-finite operand is detected by the caller
// (finite() of its own increment), since fmax drops NaN.
__device__ __forceinline__ double stage_group_max(double x) {
  x = fmax(x, dpp_double<0xB1>(x));
  x = fmax(x, dpp_double<0x4E>(x));
  return fmax(x, dpp_double<0x141>(x));
}

// Orders this lane's LDS writes before the reads that follow (in-wavefront
// exchange between the stage lanes of a body).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Own stage of the initial guess (eq. IRK_init2): L0_j = h b_j (v + sum_i nu_ji
// Rp_i) for all j, then Q_s = q + sum_j mu_sj L0_j; the same operations as the
// all-stage form, evaluated for one s (the fused mode uses the folded matrix K
// as initial_guess does).
template <bool EXACT>
__device__ __forceinline__ double stage_guess(ConstTab T, int s, double q, double v,
                                              const double (&Rp)[kS], double h) {
  if constexpr (!EXACT) {
    double acc = T[kTabC + s] * v;
#pragma unroll
    for (int j = 0; j < kS; ++j) acc = fma(T[kTabK + s * kS + j], Rp[j], acc);
    return fma(h, acc, q);
  }
  double L0[kS];
#pragma unroll
  for (int j = 0; j < kS; ++j) {
    const ConstTab r = row_tab(T);
    const double hb = h * r[kTabB + j];
    L0[j] = hb * (v + row_dot<EXACT>(r, kTabNu + j * kS, Rp));
  }
  return q + row_dot<EXACT>(T, kTabMu + s * kS, L0);
}

// Stage value q + h (c_s v + sum_j eta_sj R_j) with the coefficient row in
// registers; same operation order as stage_value.
template <bool EXACT>
__device__ __forceinline__ double stage_value_row(const double (&eta)[kS], double cs, double q,
                                                  double v, double h, const double (&R)[kS]) {
  if constexpr (EXACT) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < kS; ++j) s = s + eta[j] * R[j];
    return q + h * (cs * v + s);
  } else {
    double acc = cs * v;
#pragma unroll
    for (int j = 0; j < kS; ++j) acc = fma(eta[j], R[j], acc);
    return fma(h, acc, q);
  }
}

template <bool EXACT, int D, int NPMAX>
__global__ __launch_bounds__(8 * NPMAX) void stage_kernel(LaunchArgs a, int np) {
  constexpr int P = stage_pad<D>();
  extern __shared__ double lds[];
  double* Qt = lds;                            // [2][np][8][P]
  double* Rt = Qt + (size_t)2 * np * kS * P;   // [np][8][P]
  double* Ms = Rt + (size_t)np * kS * P;       // [np]
  int32_t* ctl = reinterpret_cast<int32_t*>(Ms + np);  // [0] instance, [1..3] notok, [4..6] bad

  const int tid = threadIdx.x;
  const int s = tid & (kS - 1);
  const int u = tid >> 3;
  const ConstTab T = const_tab(a.tab);

  // Coefficients of this lane's stage.
  double eta[kS];
#pragma unroll
  for (int j = 0; j < kS; ++j) eta[j] = a.tab[kTabEta + s * kS + j];
  const double cs = a.tab[kTabC + s];
  const double bs = a.tab[kTabB + s];

  // Promoted instances bound the length of their chunk: their wavefronts
  // take issue priority over the few-body kernel's on the same SIMDs.
  if (a.promoted) __builtin_amdgcn_s_setprio(3);
  if (tid < 7) ctl[tid] = 0;
  int64_t gk = 0;  // iteration counter over the whole launch (flag rotation)

  for (int round = 0;; ++round) {
    __syncthreads();  // the previous system is completely done with the tiles
    if (tid == 0) {
      int id = -1;
      if (a.queue_head) {
        const int idx = atomicAdd(a.queue_head, 1);
        if (idx < queue_length(a)) id = a.queue[idx];
      } else if (round == 0 && (int)blockIdx.x < a.queue_len) {
        id = a.queue[blockIdx.x];
      }
      ctl[0] = id;
    }
    __syncthreads();
    const int inst = __builtin_amdgcn_readfirstlane(ctl[0]);
    if (inst < 0) break;

    const InstDesc& dsc = a.desc[inst];
    const InstStat st0 = a.stat[inst];
    const int n = dsc.n;
    const int dq = n * D;
    const double h = dsc.h;
    const double G = dsc.G;
    const double eps2 = dsc.eps * dsc.eps;
    const int64_t stride = dsc.stride, out_off = dsc.out_off, iters_off = dsc.iters_off;
    int64_t step = st0.steps_done;
    const int64_t target = launch_target(a, step, dsc.nsteps, st0.status);
    int64_t it_sum = st0.iterations, nonconv = st0.nonconv;
    int32_t maxk = st0.max_k;
    int32_t status = st0.status;
    const bool mine = u < n;
    double* Sp = a.state + dsc.state_off;
    const double mown = (mine && dsc.mass_off >= 0) ? a.params[dsc.mass_off + u] : 1.0;

    double qh[D], ql[D], vh[D], vl[D], Qo[D], mind[D], prv[D];
#pragma unroll
    for (int d = 0; d < D; ++d) qh[d] = ql[d] = vh[d] = vl[d] = Qo[d] = mind[d] = prv[d] = 0.0;
    int buf = 0;
    if (mine && step < target) {
      if (s == 0) Ms[u] = mown;
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const int c = u * D + d;
        qh[d] = Sp[c];
        ql[d] = Sp[dq + c];
        vh[d] = Sp[2 * dq + c];
        vl[d] = Sp[3 * dq + c];
        Rt[(u * kS + s) * P + d] = Sp[4 * dq + c * kS + s];
      }
      wave_lds_sync();
#pragma unroll
      for (int d = 0; d < D; ++d) {
        double Rp[kS];
#pragma unroll
        for (int j = 0; j < kS; ++j) Rp[j] = Rt[(u * kS + j) * P + d];
        Qo[d] = stage_guess<EXACT>(T, s, qh[d], vh[d], Rp, h);
        Qt[((size_t)u * kS + s) * P + d] = Qo[d];
      }
    }

    while (step < target) {
#pragma unroll
      for (int d = 0; d < D; ++d) mind[d] = prv[d] = __builtin_inf();
      __syncthreads();  // stage positions of this step's first iteration published
      int k = 0;
      bool bad = false, capped = false;
      for (;;) {
        ++k;
        ++gk;
        if (tid == 0) {
          ctl[1 + (int)((gk + 1) % 3)] = 0;
          ctl[4 + (int)((gk + 1) % 3)] = 0;
        }
        if (mine) {
          // ---- force at this lane's stage, sources ascending
          const double* Qb = Qt + (size_t)buf * np * kS * P + s * P;
          double acc[D];
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d] = 0.0;
#pragma unroll 2
          for (int b = 0; b < n; ++b) {
            double dx[D];
#pragma unroll
            for (int d = 0; d < D; ++d) dx[d] = Qb[(size_t)b * kS * P + d] - Qo[d];
            const double mb = Ms[b];
            double r2;
            if constexpr (EXACT) {
              r2 = 0.0;
#pragma unroll
              for (int d = 0; d < D; ++d) r2 = r2 + dx[d] * dx[d];
              r2 = r2 + eps2;
            } else {
              r2 = fma(dx[0], dx[0], eps2);
#pragma unroll
              for (int d = 1; d < D; ++d) r2 = fma(dx[d], dx[d], r2);
            }
            // the self term contributes w * 0 = 0; its r2 is replaced so that
            // an unsoftened self distance does not produce 0 * inf
            r2 = (b == u) ? 1.0 : r2;
            const double w = pair_weight<EXACT>(r2, mb);
#pragma unroll
            for (int d = 0; d < D; ++d) {
              if constexpr (EXACT)
                acc[d] = acc[d] + w * dx[d];
              else
                acc[d] = fma(w, dx[d], acc[d]);
            }
          }
          const double hb = h * bs;
          double R[D];
#pragma unroll
          for (int d = 0; d < D; ++d) {
            if constexpr (EXACT)
              R[d] = hb * (G * acc[d]);
            else
              R[d] = (hb * G) * acc[d];
            Rt[(u * kS + s) * P + d] = R[d];
          }
          wave_lds_sync();
          // ---- stage update, increment and stopping rule
          double* Qn_t = Qt + (size_t)(buf ^ 1) * np * kS * P;
          bool ok = true, nf = false;
#pragma unroll
          for (int d = 0; d < D; ++d) {
            double Rj[kS];
#pragma unroll
            for (int j = 0; j < kS; ++j) Rj[j] = Rt[(u * kS + j) * P + d];
            const double qn = stage_value_row<EXACT>(eta, cs, qh[d], vh[d], h, Rj);
            const double dd = fabs(qn - Qo[d]);
            nf |= !finite(dd);
            const double dmax = stage_group_max(dd);
            Qo[d] = qn;
            Qn_t[((size_t)u * kS + s) * P + d] = qn;
            ok &= stop_component(dmax, mind[d], prv[d]);
          }
          if (!ok) ctl[1 + (int)(gk % 3)] = 1;
          if (nf) ctl[4 + (int)(gk % 3)] = 1;
        }
        __syncthreads();
        const int notok = __builtin_amdgcn_readfirstlane(ctl[1 + (int)(gk % 3)]);
        const int badf = __builtin_amdgcn_readfirstlane(ctl[4 + (int)(gk % 3)]);
        buf ^= 1;
        if (badf) {
          bad = true;
          break;
        }
        if (!notok) break;
        if (k >= a.max_iter) {
          capped = true;
          break;
        }
      }

      // ---- end of step
      if (bad) {
        if (mine && s == 0) {
          const int64_t nfr = target / stride;  // frames of this launch only
          for (int64_t f = step / stride + 1; f <= nfr; ++f)
#pragma unroll
            for (int d = 0; d < D; ++d) {
              a.qout[out_off + f * dq + u * D + d] = __builtin_nan("");
              a.pout[out_off + f * dq + u * D + d] = __builtin_nan("");
            }
        }
        if (tid == 0 && iters_off >= 0) a.step_iters[iters_off + step] = (uint8_t)k;
        status = kNonFinite;
        break;
      }
      if (tid == 0 && iters_off >= 0) a.step_iters[iters_off + step] = (uint8_t)k;
      ++step;
      it_sum += k;
      nonconv += capped ? 1 : 0;
      maxk = k > maxk ? k : maxk;
      const bool frame = (step % stride) == 0;
      const bool last = step >= target;
      if (mine) {
        const ConstTab r = row_tab(T);
        const double Rown[3] = {D > 0 ? Rt[(u * kS + s) * P + 0] : 0.0,
                                D > 1 ? Rt[(u * kS + s) * P + 1] : 0.0,
                                D > 2 ? Rt[(u * kS + s) * P + 2] : 0.0};
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int c = u * D + d;
          double Rj[kS];
#pragma unroll
          for (int j = 0; j < kS; ++j) Rj[j] = Rt[(u * kS + j) * P + d];
          double sv, sc;
          step_sums<EXACT>(r, Rj, sv, sc);
          dw_add(vh[d], vl[d], sv);
          dw_add(qh[d], ql[d], h * (vh[d] - sc));
          if (s == 0) {
            if (frame) {
              const int64_t f = step / stride;
              a.qout[out_off + f * dq + c] = qh[d];
              a.pout[out_off + f * dq + c] = mown * vh[d];
            }
            if (last) {
              Sp[c] = qh[d];
              Sp[dq + c] = ql[d];
              Sp[2 * dq + c] = vh[d];
              Sp[3 * dq + c] = vl[d];
            }
          }
          if (last) {
            Sp[4 * dq + c * kS + s] = Rown[d];
          } else {
            Qo[d] = stage_guess<EXACT>(T, s, qh[d], vh[d], Rj, h);
            Qt[((size_t)buf * np * kS + u * kS + s) * P + d] = Qo[d];
          }
        }
      }
    }
    if (tid == 0) {
      InstStat st;
      st.steps_done = step;
      st.iterations = it_sum;
      st.nonconv = nonconv;
      st.max_k = maxk;
      st.status = status;
      a.stat[inst] = st;
    }
  }
}

// ------------------------------------------------------------------ launchers

bool stage_class_supported(int kind, int n, int d) {
  return kind == kGravity && d >= 1 && d <= 3 && n >= 1 && n <= kStageMaxBodies;
}

// Padded body count (multiple of 8, so 8 np lanes fill whole wavefronts).
int stage_np(int n) { return (n + 7) / 8 * 8; }

template <bool EXACT, int D, int NPMAX>
static hipError_t launch_stage_t(const LaunchArgs& a, int np, int n_items, int num_cus,
                                 hipStream_t st) {
  auto kern = stage_kernel<EXACT, D, NPMAX>;
  const size_t lds = sizeof(double) * stage_lds_doubles<D>(np) + 8 * sizeof(int32_t);
  hipError_t e =
      hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int TT = kS * np;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TT, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int cap = class_blocks_per_cu(per_cu, TT / 64) * num_cus;
  const int grid = n_items < cap ? n_items : cap;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(TT), lds, st, a, np);
  return hipGetLastError();
}

template <bool EXACT, int D>
static hipError_t launch_stage_d(const LaunchArgs& a, int np, int n_items, int num_cus,
                                 hipStream_t st) {
  if (np <= 16) return launch_stage_t<EXACT, D, 16>(a, np, n_items, num_cus, st);
  if (np <= 32) return launch_stage_t<EXACT, D, 32>(a, np, n_items, num_cus, st);
  if (np <= 64) return launch_stage_t<EXACT, D, 64>(a, np, n_items, num_cus, st);
  return launch_stage_t<EXACT, D, 128>(a, np, n_items, num_cus, st);
}

// Class key: (gravity, d, np).  n_items instances, all with padded size np.
hipError_t launch_stage_class(int d, int np, const LaunchArgs& a, int n_items, int num_cus,
                              hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (np < 8 || np > kStageMaxBodies || np % 8 != 0) return hipErrorInvalidValue;
  const bool ex = a.exact != 0;
  switch (d) {
    case 1: return ex ? launch_stage_d<true, 1>(a, np, n_items, num_cus, st)
                      : launch_stage_d<false, 1>(a, np, n_items, num_cus, st);
    case 2: return ex ? launch_stage_d<true, 2>(a, np, n_items, num_cus, st)
                      : launch_stage_d<false, 2>(a, np, n_items, num_cus, st);
    case 3: return ex ? launch_stage_d<true, 3>(a, np, n_items, num_cus, st)
                      : launch_stage_d<false, 3>(a, np, n_items, num_cus, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace irk

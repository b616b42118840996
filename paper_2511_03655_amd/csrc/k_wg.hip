// Persistent batched IRKGL16 kernel for larger systems: gravitational systems
// of up to 512 bodies (Plummer clusters, planetary systems with many bodies)
// and FPU-beta chains of up to 1024 sites.
//
// Mapping: one lane owns one body (d = 3) or chain site (d = 1) with all 8
// stage values of its components in registers, so the 8x8 stage contraction
// Q_i = q + h (c_i v + sum_j eta_ij R_j) (eq. IRK_FP2), the max-norm increment
// and stopping rule (eqs. Delta_n, stopping), the compensated update
// (eq. qnvn2) and the extrapolated initial guess (eq. IRK_init2) are all
// lane-local.  The force needs the other bodies' (or the neighbours') stage
// positions: each iteration the lanes publish their 8 x d stage positions to an
// LDS tile laid out [unit][stage][component] (units an odd number of doubles
// apart), and every lane reads the source units it needs from there (gravity:
// all bodies of its system, summed in ascending order; chain: the two
// neighbours).
//
// A workgroup of T lanes is split into T / S slots of S lanes (S >= n, one
// system per slot); slots iterate in lockstep, converged slots are masked, and
// a slot whose system finishes pulls the next one from the class queue.  Per
// system arithmetic does not depend on the slot or workgroup that runs it.
#include "device_common.h"
#include "pair_weight.h"

namespace irk {

// Doubles per unit in the stage tile: the unit's 8 x D stage positions plus
// one pad, so that consecutive lanes' units start an odd number of doubles
// apart.  A stride of 8 D doubles (a multiple of 16 four-byte banks) would put
// the 16 lanes of one 64-bit LDS pass on two banks when each lane reads or
// writes its own unit, or a neighbour's.
template <int D>
constexpr int wg_unit_stride() {
  static_assert((kS * D + 1) % 2 == 1, "odd unit stride");
  return kS * D + 1;
}

struct WgMeta {
  int64_t nsteps, stride, out_off, iters_off, state_off, step, target, it_sum, nonconv;
  double h, G, eps2, beta;
  int32_t inst, n, maxk, kslot, flags, notok, bad, pad;
};

template <int KIND, int D, bool EXACT>
__device__ __forceinline__ void unit_increments(const double* __restrict__ Qs,
                                                const double* __restrict__ Ms, int base, int u,
                                                int n, const WgMeta& M, double kl, double kr,
                                                ConstTab T, double h, double (&R)[D][kS],
                                                int b_lo, int b_hi) {
  // The lane's own stage positions are read back from the tile (it published
  // them there), so they need not stay in registers across the force loop.
  constexpr int US = wg_unit_stride<D>();
  const double* qa = Qs + (size_t)(base + u) * US;
  if constexpr (KIND == kGravity) {
    // Sources b ascending; the 8 stages of a source are 8 independent chains
    // (instruction-level parallelism); each stage's sum keeps the b order.
    const double eps2 = M.eps2;
    double acc[D][kS] = {};
    for (int b = b_lo; b < b_hi; ++b) {
      if (b == u) continue;
      const double* qb = Qs + (size_t)(base + b) * US;
      const double mb = Ms[base + b];
#pragma unroll
      for (int s = 0; s < kS; ++s) {
        double dx[D];
#pragma unroll
        for (int d = 0; d < D; ++d) dx[d] = qb[s * D + d] - qa[s * D + d];
        if constexpr (EXACT) {
          double r2 = 0.0;
#pragma unroll
          for (int d = 0; d < D; ++d) r2 = r2 + dx[d] * dx[d];
          r2 = r2 + eps2;
          const double w = pair_weight<true>(r2, mb);
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d][s] = acc[d][s] + w * dx[d];
        } else {
          double r2 = fma(dx[0], dx[0], eps2);
#pragma unroll
          for (int d = 1; d < D; ++d) r2 = fma(dx[d], dx[d], r2);
          const double w = mass_rinv3_halley(r2, mb);
#pragma unroll
          for (int d = 0; d < D; ++d) acc[d][s] = fma(w, dx[d], acc[d][s]);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kS; ++s) {
      const double hb = h * T[kTabB + s];
#pragma unroll
      for (int d = 0; d < D; ++d) {
        if constexpr (EXACT)
          R[d][s] = hb * (M.G * acc[d][s]);
        else
          R[d][s] = (hb * M.G) * acc[d][s];
      }
    }
  } else {  // chain, D == 1: F = k_r V'(q_{i+1} - q_i) - k_l V'(q_i - q_{i-1})
    const double beta = M.beta;
    const double m_site = Ms[base + u];
#pragma unroll
    for (int s = 0; s < kS; ++s) {
      const double ql = (u > 0) ? Qs[(size_t)(base + u - 1) * US + s] : 0.0;
      const double qr = (u < n - 1) ? Qs[(size_t)(base + u + 1) * US + s] : 0.0;
      const double sr = qr - qa[s];
      const double sl = qa[s] - ql;
      double F;
      if constexpr (EXACT) {
        F = kr * (sr + beta * (sr * sr * sr)) - kl * (sl + beta * (sl * sl * sl));
      } else {
        const double vr = fma(beta * sr * sr, sr, sr);
        const double vl = fma(beta * sl * sl, sl, sl);
        F = fma(kr, vr, -(kl * vl));
      }
      R[0][s] = (h * T[kTabB + s]) * (F / m_site);
    }
  }
}

// SPLIT (gravity, fast mode, systems of up to 256 bodies): a slot of S lanes
// holds one system on S / 2 body lanes; lane u >= S / 2 helps body u - S / 2 by
// summing the upper half of the sources (b >= ceil(n / 2)) while the body lane
// sums the lower half, and passes its increments through its own row of the
// stage tile (no body's unit lives there); the body lane's increment is the
// sum lower + upper.  A lone system of 256 bodies then keeps two wavefronts
// per SIMD busy instead of one (one wavefront alone issues FP64 work at about
// half the SIMD's rate).  Arithmetic per system still depends on its size
// only.
template <int KIND, int D, bool EXACT, int MAXT, bool SPLIT>
__global__ __launch_bounds__(MAXT) void wg_kernel(LaunchArgs a, int S) {
  extern __shared__ double lds[];
  const int TT = blockDim.x;
  const int nslots = TT / S;
  double* Qs = lds;                                  // [TT][8 D + 1]
  constexpr int US = wg_unit_stride<D>();
  double* Ms = Qs + (size_t)TT * US;                 // [TT] masses of the units
  WgMeta* meta = reinterpret_cast<WgMeta*>(Ms + TT);  // [nslots]
  int32_t* slot_inst = reinterpret_cast<int32_t*>(meta + nslots);
  int32_t* qdone = slot_inst + nslots;

  const int tid = threadIdx.x;
  const int slot = tid / S;
  const int us = tid - slot * S;            // lane within the slot
  const int Sb = SPLIT ? S / 2 : S;         // body lanes of the slot
  const bool helper = SPLIT && us >= Sb;    // sums the upper half of the sources
  const int u = helper ? us - Sb : us;      // body of this lane
  const int base = slot * S;
  WgMeta& M = meta[slot];
  const ConstTab T = const_tab(a.tab);

  int inst = -1;
  double qh[D] = {}, ql[D] = {}, vh[D] = {}, vl[D] = {}, mind[D] = {}, prv[D] = {};
  double Q[D][kS] = {}, R[D][kS] = {};
  double mown = 1.0, kl = 1.0, kr = 1.0;

  if (tid == 0) *qdone = 0;
  if (tid < nslots) {
    slot_inst[tid] = -1;
    meta[tid].inst = -1;
  }
  __syncthreads();

  for (;;) {
    if (us == 0 && slot_inst[slot] < 0 && !*qdone) {
      if (a.queue_head) {
        const int idx = atomicAdd(a.queue_head, 1);
        if (idx < queue_length(a))
          slot_inst[slot] = a.queue[idx];
        else
          *qdone = 1;
      } else if (slot < a.queue_len) {
        slot_inst[slot] = a.queue[slot];
      }
    }
    __syncthreads();
    if (!a.queue_head && tid == 0) *qdone = 1;
    const int cur = slot_inst[slot];
    if (__syncthreads_or(cur >= 0) == 0) break;

    const bool fresh = cur >= 0 && cur != inst;
    if (fresh && us == 0) {
      const InstDesc& dsc = a.desc[cur];
      const InstStat st = a.stat[cur];
      M.inst = cur;
      M.n = dsc.n;
      M.h = dsc.h;
      M.G = dsc.G;
      M.eps2 = dsc.eps * dsc.eps;
      M.beta = dsc.beta;
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
    }
    __syncthreads();
    const int n = (cur >= 0) ? M.n : 0;
    const bool mine = u < n && !helper;  // this lane owns a unit of the slot's system
    const bool forces = u < n;           // this lane sums forces on unit u
    const int nh = SPLIT ? (n + 1) / 2 : n;
    const int b_lo = helper ? nh : 0, b_hi = (SPLIT && !helper) ? nh : n;
    if (fresh) {
      inst = cur;
      const InstDesc& dsc = a.desc[cur];
      if (mine) {
        mown = (dsc.mass_off >= 0) ? a.params[dsc.mass_off + u] : 1.0;
        if constexpr (KIND == kChain) {
          kl = (dsc.coupling_off >= 0) ? a.params[dsc.coupling_off + u] : 1.0;
          kr = (dsc.coupling_off >= 0) ? a.params[dsc.coupling_off + u + 1] : 1.0;
        }
        Ms[base + u] = mown;
        const int dq = n * D;
        const double* Sp = a.state + M.state_off;
        double Rp[D][kS];
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const int c = u * D + d;
          qh[d] = Sp[c];
          ql[d] = Sp[dq + c];
          vh[d] = Sp[2 * dq + c];
          vl[d] = Sp[3 * dq + c];
#pragma unroll
          for (int s = 0; s < kS; ++s) Rp[d][s] = Sp[4 * dq + c * kS + s];
        }
        initial_guess<D, EXACT>(T, qh, vh, Rp, M.h, Q);
      }
    }

    // ---- one step, all live slots in lockstep.  The stage positions are
    // published to the tile before the first iteration and right after each
    // update (behind the barrier that ends the force reads), so Q is only live
    // between an update and its publication.
    const bool live = (inst >= 0) && (M.step < M.target);
    const double h = M.h;
    bool conv = !live;
#pragma unroll
    for (int d = 0; d < D; ++d) mind[d] = prv[d] = __builtin_inf();
    if (!conv && mine) {
#pragma unroll
      for (int s = 0; s < kS; ++s)
#pragma unroll
        for (int d = 0; d < D; ++d) Qs[(size_t)(base + u) * US + s * D + d] = Q[d][s];
    }
    int k = 0;
    while (__syncthreads_or(!conv)) {
      ++k;
      if (!conv && us == 0) {
        M.notok = 0;
        M.bad = 0;
      }
      __syncthreads();
      double Qn[D][kS] = {};
      if (!conv && forces)
        unit_increments<KIND, D, EXACT>(Qs, Ms, base, u, n, M, kl, kr, T, h, R, b_lo, b_hi);
      if constexpr (SPLIT) {
        // the helper's increments go to its own tile row; the body lane adds them
        double* row = Qs + (size_t)(base + Sb + u) * US;
        if (!conv && forces && helper) {
#pragma unroll
          for (int s = 0; s < kS; ++s)
#pragma unroll
            for (int d = 0; d < D; ++d) row[s * D + d] = R[d][s];
        }
        __syncthreads();
        if (!conv && mine) {
#pragma unroll
          for (int s = 0; s < kS; ++s)
#pragma unroll
            for (int d = 0; d < D; ++d) R[d][s] = R[d][s] + row[s * D + d];
        }
      }
      if (!conv && mine) {
        const double* qa = Qs + (size_t)(base + u) * US;
        bool ok = true, bad = false;
        double dmax[D], nf[D];
#pragma unroll
        for (int d = 0; d < D; ++d) dmax[d] = nf[d] = 0.0;
#pragma unroll
        for (int s = 0; s < kS; ++s) {
          const ConstTab r = row_tab(T);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            Qn[d][s] = stage_value<EXACT>(r, s, qh[d], vh[d], h, R[d]);
            max_track(dmax[d], nf[d], fabs(Qn[d][s] - qa[s * D + d]));
          }
        }
#pragma unroll
        for (int d = 0; d < D; ++d) {
          bad |= !track_finite(dmax[d], nf[d]);
          ok &= stop_component(dmax[d], mind[d], prv[d]);
        }
        if (!ok) M.notok = 1;
        if (bad) M.bad = 1;
      }
      __syncthreads();
      if (!conv) {
        const bool slot_bad = M.bad != 0;
        const bool slot_ok = M.notok == 0;
        if (slot_ok || slot_bad || k >= a.max_iter) {
          conv = true;
          if (us == 0) {
            M.kslot = k;
            M.flags = (slot_bad ? 1 : 0) | ((!slot_ok && !slot_bad) ? 2 : 0);
          }
        } else if (mine) {
#pragma unroll
          for (int s = 0; s < kS; ++s)
#pragma unroll
            for (int d = 0; d < D; ++d) Qs[(size_t)(base + u) * US + s * D + d] = Qn[d][s];
        }
      }
    }
    __syncthreads();

    // ---- end of step
    bool release = (inst >= 0) && !live;
    if (live) {
      const int kslot = M.kslot;
      const int64_t step0 = M.step, stride = M.stride, out_off = M.out_off;
      const int dq = n * D;
      if (M.flags & 1) {
        if (mine) {
          const int64_t nf = M.target / stride;  // frames of this launch only
          for (int64_t f = step0 / stride + 1; f <= nf; ++f)
#pragma unroll
            for (int d = 0; d < D; ++d) {
              a.qout[out_off + f * dq + u * D + d] = __builtin_nan("");
              a.pout[out_off + f * dq + u * D + d] = __builtin_nan("");
            }
        }
        if (us == 0) {
          if (M.iters_off >= 0) a.step_iters[M.iters_off + step0] = (uint8_t)kslot;
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
        if (mine) {
          double* Sp = a.state + M.state_off;
          const ConstTab r = row_tab(T);
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const int c = u * D + d;
            double sv, sc;
            step_sums<EXACT>(r, R[d], sv, sc);
            dw_add(vh[d], vl[d], sv);
            dw_add(qh[d], ql[d], h * (vh[d] - sc));
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
#pragma unroll
              for (int s = 0; s < kS; ++s) Sp[4 * dq + c * kS + s] = R[d][s];
            }
          }
          if (!last) initial_guess<D, EXACT>(T, qh, vh, R, h, Q);
        }
        if (us == 0) {
          if (M.iters_off >= 0) a.step_iters[M.iters_off + step0] = (uint8_t)kslot;
          M.step = step;
          M.it_sum += kslot;
          M.nonconv += (M.flags & 2) ? 1 : 0;
          if (kslot > M.maxk) M.maxk = kslot;
          if (last) {
            InstStat st;
            st.steps_done = step;
            st.iterations = M.it_sum;
            st.nonconv = M.nonconv;
            st.max_k = M.maxk;
            st.status = kOk;
            a.stat[inst] = st;
          }
        }
        release = last;
      }
    }
    __syncthreads();
    if (release) {
      if (us == 0) slot_inst[slot] = -1;
      inst = -1;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ launchers

// Largest system (bodies or sites) the workgroup kernel accepts per kind.
constexpr int kWgMaxGravity = 512;
constexpr int kWgMaxChain = 1024;

// Slot width for a system of n units: a power of two up to 64, else a multiple
// of 64.
int wg_slot_size(int n) {
  if (n <= 64) {
    int s = 8;
    while (s < n) s <<= 1;
    return s;
  }
  return (n + 63) / 64 * 64;
}

int wg_block_size(int S) { return S <= 256 ? 256 : (S <= 512 ? 512 : 1024); }

size_t wg_lds_bytes(int TT, int S, int D) {
  const int nslots = TT / S;
  const int us = kS * D + 1;  // wg_unit_stride<D>()
  return sizeof(double) * ((size_t)TT * us + TT) + sizeof(WgMeta) * nslots +
         sizeof(int32_t) * (nslots + 1);
}

bool wg_class_supported(int kind, int n, int d) {
  if (kind == kGravity) return d == 3 && n >= 1 && n <= kWgMaxGravity;
  if (kind == kChain) return d == 1 && n >= 1 && n <= kWgMaxChain;
  return false;
}

template <int KIND, int D>
hipError_t launch_wg(const LaunchArgs& a, int S, int n_items, int num_cus, hipStream_t st,
                     int block) {
  constexpr int MAXT = (KIND == kGravity) ? 512 : 1024;
  // gravity in the fast mode up to 256 bodies: two lanes per body (SPLIT), so
  // the slot is twice the body slot
  const bool split = KIND == kGravity && !a.exact && 2 * S <= MAXT;
  if (split) S *= 2;
  // tuned block: a multiple of the slot width and of 64, at least the slot
  const int TT = (block >= S && block % S == 0 && block % 64 == 0 && block <= MAXT)
                     ? block
                     : wg_block_size(S);
  const size_t lds = wg_lds_bytes(TT, S, D);
  if (TT > MAXT) return hipErrorInvalidConfiguration;
  auto kern = a.exact ? wg_kernel<KIND, D, true, MAXT, false>
                      : (split ? wg_kernel<KIND, D, false, MAXT, KIND == kGravity>
                               : wg_kernel<KIND, D, false, MAXT, false>);
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  int per_cu = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, TT, lds);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorInvalidConfiguration;
  const int nslots = TT / S;
  const int want = (n_items + nslots - 1) / nslots;
  const int cap = class_blocks_per_cu(per_cu, TT / 64) * num_cus;
  const int grid = want < cap ? want : cap;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(TT), lds, st, a, S);
  return hipGetLastError();
}

// Class key: (kind, d, S).  n_items instances, all with slot size S.
hipError_t launch_wg_class(int kind, int d, int S, const LaunchArgs& a, int n_items, int num_cus,
                           hipStream_t st, int block) {
  if (n_items <= 0) return hipSuccess;
  if (kind == kGravity && d == 3) return launch_wg<kGravity, 3>(a, S, n_items, num_cus, st, block);
  if (kind == kChain && d == 1) return launch_wg<kChain, 1>(a, S, n_items, num_cus, st, block);
  return hipErrorInvalidValue;
}

}  // namespace irk

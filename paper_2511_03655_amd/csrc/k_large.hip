// IRKGL16 for one large gravitational system (N > 512 bodies, e.g. a 2048-body
// Plummer cluster): the whole GPU works on one system.
//
// One cooperative persistent launch per integration call.  Workgroups are
// (stage s, block of 256 targets, source chunk c).  Per fixed-point iteration:
//  * force: each workgroup stages its chunk of source positions at stage s in
//    LDS and accumulates, for its 256 targets, sum_b m_b (q_b - q_a) r^-3 over
//    the chunk (sources ascending); partial sums go to HBM;
//  * update: the last workgroup to finish a target block (atomic arrival
//    counter with release/acquire fences) sums the chunk partials in chunk order,
//    forms R_i = h b_i G g_i, the new stage values (eq. IRK_FP2), the per
//    component max-norm increment and the stopping rule (eqs. Delta_n,
//    stopping) for that block, and raises a global "not converged" flag;
//  * one grid barrier, then every workgroup reads the flag.
// Stage positions are double-buffered by iteration parity (a block may be
// updated while other blocks still read the previous positions); flags rotate
// over three slots so that a reset never races a reader.  After convergence the
// component lanes perform the compensated update (eq. qnvn2), outputs and the
// next initial guess (eq. IRK_init2); one more grid barrier ends the step.
// With EXACT (reproducible mode) a single chunk is used, so every sum runs in
// the reference order.
#include <hip/hip_cooperative_groups.h>

#include "device_common.h"

namespace cg = cooperative_groups;

namespace irk {

struct LargeArgs {
  LaunchArgs a;
  int32_t inst;       // instance id
  int32_t n;          // bodies
  int32_t nchunks;    // source chunks
  int32_t ntb;        // target blocks of 256
  double* pos;        // [2][8][n][3]
  double* part;       // [nchunks][8][n][3]
  double* rbuf;       // [3n][8]   increments R of the last iteration
  double* hist;       // [3n][2]   mind, prev
  int32_t* arrive;    // [ntb]     arrival counters
  int32_t* flags;     // [3][2]    notok, bad by iteration % 3
  int64_t* ctl;       // [4]       scratch for the final statistics
};

constexpr int kLargeBlock = 256;
constexpr int kLargeTile = 1024;  // sources staged in LDS at a time

template <bool EXACT>
__global__ __launch_bounds__(kLargeBlock) void large_kernel(LargeArgs L) {
  cg::grid_group grid = cg::this_grid();
  const LaunchArgs& a = L.a;
  const ConstTab T = const_tab(a.tab);
  const InstDesc dsc = a.desc[L.inst];
  const int n = L.n;
  const int dq = 3 * n;
  const int tid = threadIdx.x;
  const int bid = blockIdx.x;
  const int nblocks = gridDim.x;
  // block -> (stage, target block, chunk)
  const int s = bid % kS;
  const int tb = (bid / kS) % L.ntb;
  const int c = bid / (kS * L.ntb);
  const int chunk = (n + L.nchunks - 1) / L.nchunks;
  const int src0 = c * chunk;
  const int src1 = min(n, src0 + chunk);
  const int tgt = tb * kLargeBlock + tid;
  const int gtid = bid * kLargeBlock + tid;  // component lane for the step end

  __shared__ double src[kLargeTile * 3];
  __shared__ double msrc[kLargeTile];
  __shared__ int32_t last_flag;

  const double* mass = a.params + dsc.mass_off;
  double* S = a.state + dsc.state_off;
  const double h = dsc.h;
  const double G = dsc.G;
  const double eps2 = dsc.eps * dsc.eps;
  const InstStat st0 = a.stat[L.inst];
  int64_t step = st0.steps_done;
  int64_t target = dsc.nsteps;
  if (a.step_budget > 0 && step + a.step_budget < dsc.nsteps) target = step + a.step_budget;
  if (st0.status != kOk) target = step;
  int64_t it_sum = st0.iterations, nonconv = st0.nonconv;
  int32_t maxk = st0.max_k;
  bool dead = false;
  int64_t it = 0;  // global iteration counter (parity of the position buffers)

  // Initial guess of the first step from the stored state, into pos[0].
  if (gtid < dq && step < target) {
    const double qh = S[gtid], vh = S[2 * dq + gtid];
    double Rp[1][kS], Q0[1][kS];
#pragma unroll
    for (int j = 0; j < kS; ++j) Rp[0][j] = S[4 * dq + gtid * kS + j];
    const double qa[1] = {qh}, va[1] = {vh};
    initial_guess<1, EXACT>(T, qa, va, Rp, h, Q0);
    const int body = gtid / 3, d = gtid % 3;
#pragma unroll
    for (int j = 0; j < kS; ++j) L.pos[((size_t)j * n + body) * 3 + d] = Q0[0][j];
    L.hist[2 * gtid] = __builtin_inf();
    L.hist[2 * gtid + 1] = __builtin_inf();
  }
  if (bid == 0 && tid < 9) L.flags[tid] = 0;
  if (bid == 0 && tid == 0) {
    for (int t = 0; t < L.ntb; ++t) L.arrive[t] = 0;
  }
  grid.sync();

  while (step < target && !dead) {
    int k = 0;
    bool conv = false, capped = false;
    for (;;) {
      ++k;
      const double* P = L.pos + (size_t)(it & 1) * kS * n * 3;
      double* Pn = L.pos + (size_t)((it + 1) & 1) * kS * n * 3;
      const int fl = (int)(it % 3);
      // ---- force partial sums for (stage s, targets of block tb, chunk c)
      double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
      double qa0 = 0.0, qa1 = 0.0, qa2 = 0.0;
      if (tgt < n) {
        qa0 = P[((size_t)s * n + tgt) * 3 + 0];
        qa1 = P[((size_t)s * n + tgt) * 3 + 1];
        qa2 = P[((size_t)s * n + tgt) * 3 + 2];
      }
      for (int t0 = src0; t0 < src1; t0 += kLargeTile) {
        const int t1 = min(src1, t0 + kLargeTile);
        __syncthreads();
        for (int b = t0 + tid; b < t1; b += kLargeBlock) {
          src[(b - t0) * 3 + 0] = P[((size_t)s * n + b) * 3 + 0];
          src[(b - t0) * 3 + 1] = P[((size_t)s * n + b) * 3 + 1];
          src[(b - t0) * 3 + 2] = P[((size_t)s * n + b) * 3 + 2];
          msrc[b - t0] = mass[b];
        }
        __syncthreads();
        if (tgt < n) {
          for (int b = t0; b < t1; ++b) {
            if (b == tgt) continue;
            const double dx = src[(b - t0) * 3 + 0] - qa0;
            const double dy = src[(b - t0) * 3 + 1] - qa1;
            const double dz = src[(b - t0) * 3 + 2] - qa2;
            if constexpr (EXACT) {
              double r2 = 0.0;
              r2 = r2 + dx * dx;
              r2 = r2 + dy * dy;
              r2 = r2 + dz * dz;
              r2 = r2 + eps2;
              const double w = pair_weight<true>(r2, msrc[b - t0]);
              acc0 = acc0 + w * dx;
              acc1 = acc1 + w * dy;
              acc2 = acc2 + w * dz;
            } else {
              const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
              const double w = msrc[b - t0] * rinv3(r2 + eps2);
              acc0 = fma(w, dx, acc0);
              acc1 = fma(w, dy, acc1);
              acc2 = fma(w, dz, acc2);
            }
          }
        }
      }
      if (tgt < n) {
        double* pp = L.part + (((size_t)c * kS + s) * n + tgt) * 3;
        pp[0] = acc0;
        pp[1] = acc1;
        pp[2] = acc2;
      }
      // ---- arrival; the last workgroup of this target block does its update
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        const int prev = atomicAdd(&L.arrive[tb], 1);
        last_flag = (prev == kS * L.nchunks - 1) ? 1 : 0;
        if (last_flag) L.arrive[tb] = 0;
      }
      __syncthreads();
      if (last_flag) {
        __threadfence();
        if (tgt < n) {
          bool ok = true, bad = false;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int comp = tgt * 3 + d;
            const double qh = S[comp], vh = S[2 * dq + comp];
            double R[kS];
#pragma unroll
            for (int j = 0; j < kS; ++j) {
              double g;
              if constexpr (EXACT) {
                g = L.part[((size_t)j * n + tgt) * 3 + d];  // single chunk
                R[j] = (h * T[kTabB + j]) * (G * g);
              } else {
                g = 0.0;
                for (int cc = 0; cc < L.nchunks; ++cc)
                  g += L.part[(((size_t)cc * kS + j) * n + tgt) * 3 + d];
                R[j] = ((h * T[kTabB + j]) * G) * g;
              }
            }
            double dmax = 0.0;
#pragma unroll
            for (int j = 0; j < kS; ++j) {
              const ConstTab r = row_tab(T);
              const double qn = stage_value<EXACT>(r, j, qh, vh, h, R);
              dmax = max_keep_nan(dmax, fabs(qn - P[((size_t)j * n + tgt) * 3 + d]));
              Pn[((size_t)j * n + tgt) * 3 + d] = qn;
            }
#pragma unroll
            for (int j = 0; j < kS; ++j) L.rbuf[(size_t)comp * kS + j] = R[j];
            double mind = L.hist[2 * comp], prv = L.hist[2 * comp + 1];
            bad |= !finite(dmax);
            ok &= stop_component(dmax, mind, prv);
            L.hist[2 * comp] = mind;
            L.hist[2 * comp + 1] = prv;
          }
          if (!ok) atomicOr(&L.flags[fl * 2 + 0], 1);
          if (bad) atomicOr(&L.flags[fl * 2 + 1], 1);
        }
      }
      // reset the flags of iteration it + 1 (last read two barriers ago)
      if (bid == 0 && tid < 2) L.flags[((it + 1) % 3) * 2 + tid] = 0;
      __threadfence();
      grid.sync();
      const int notok = __hip_atomic_load(&L.flags[fl * 2 + 0], __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
      const int badf = __hip_atomic_load(&L.flags[fl * 2 + 1], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
      ++it;
      if (badf) {
        dead = true;
        break;
      }
      if (!notok) {
        conv = true;
        break;
      }
      if (k >= a.max_iter) {
        capped = true;
        break;
      }
    }
    // ---- end of step (component lanes spread over the whole grid)
    if (dead) {
      if (gtid < dq) {
        const int64_t nf = target / dsc.stride;  // frames of this launch only
        for (int64_t f = step / dsc.stride + 1; f <= nf; ++f) {
          a.qout[dsc.out_off + f * dq + gtid] = __builtin_nan("");
          a.pout[dsc.out_off + f * dq + gtid] = __builtin_nan("");
        }
      }
      if (bid == 0 && tid == 0 && dsc.iters_off >= 0) a.step_iters[dsc.iters_off + step] = (uint8_t)k;
      break;
    }
    (void)conv;
    ++step;
    it_sum += k;
    nonconv += capped ? 1 : 0;
    maxk = k > maxk ? k : maxk;
    if (gtid < dq) {
      double qh = S[gtid], ql = S[dq + gtid], vh = S[2 * dq + gtid], vl = S[3 * dq + gtid];
      double R[1][kS];
#pragma unroll
      for (int j = 0; j < kS; ++j) R[0][j] = L.rbuf[(size_t)gtid * kS + j];
      double sv, sc;
      step_sums<EXACT>(T, R[0], sv, sc);
      dw_add(vh, vl, sv);
      dw_add(qh, ql, h * (vh - sc));
      S[gtid] = qh;
      S[dq + gtid] = ql;
      S[2 * dq + gtid] = vh;
      S[3 * dq + gtid] = vl;
#pragma unroll
      for (int j = 0; j < kS; ++j) S[4 * dq + gtid * kS + j] = R[0][j];
      if (step % dsc.stride == 0) {
        const int64_t f = step / dsc.stride;
        a.qout[dsc.out_off + f * dq + gtid] = qh;
        a.pout[dsc.out_off + f * dq + gtid] = mass[gtid / 3] * vh;
      }
      if (step < target) {
        double Q0[1][kS];
        const double qa[1] = {qh}, va[1] = {vh};
        initial_guess<1, EXACT>(T, qa, va, R, h, Q0);
        double* Pn = L.pos + (size_t)(it & 1) * kS * n * 3;
        const int body = gtid / 3, d = gtid % 3;
#pragma unroll
        for (int j = 0; j < kS; ++j) Pn[((size_t)j * n + body) * 3 + d] = Q0[0][j];
        L.hist[2 * gtid] = __builtin_inf();
        L.hist[2 * gtid + 1] = __builtin_inf();
      }
    }
    if (bid == 0 && tid == 0 && dsc.iters_off >= 0) a.step_iters[dsc.iters_off + step - 1] = (uint8_t)k;
    __threadfence();
    grid.sync();
  }
  if (bid == 0 && tid == 0) {
    InstStat st;
    st.steps_done = step;
    st.iterations = it_sum;
    st.nonconv = nonconv;
    st.max_k = maxk;
    st.status = dead ? kNonFinite : (st0.status != kOk ? st0.status : kOk);
    a.stat[L.inst] = st;
  }
  (void)nblocks;
}

bool large_class_supported(int kind, int n, int d) { return kind == kGravity && d == 3 && n > 1; }

// Device scratch needed for a system of n bodies with the given chunk count.
size_t large_scratch_bytes(int n, int nchunks) {
  const int ntb = (n + kLargeBlock - 1) / kLargeBlock;
  return sizeof(double) * ((size_t)2 * kS * n * 3 + (size_t)nchunks * kS * n * 3 +
                            (size_t)3 * n * kS + (size_t)3 * n * 2) +
         sizeof(int32_t) * (ntb + 9) + sizeof(int64_t) * 4 + 256;
}

// Chunk count: the largest power of two (<= 16, chunks of >= 64 sources) whose
// grid still fits co-resident; 1 in reproducible mode.
int large_chunks(int n, bool exact, int num_cus) {
  if (exact) return 1;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, large_kernel<false>, kLargeBlock, 0) !=
          hipSuccess ||
      per_cu < 1)
    return 1;
  const int ntb = (n + kLargeBlock - 1) / kLargeBlock;
  int ch = 1;
  while (ch < 16 && n / (2 * ch) >= 64 && kS * ntb * (2 * ch) <= per_cu * num_cus) ch *= 2;
  return ch;
}

hipError_t launch_large(const LaunchArgs& a, int inst, int n, void* scratch, int nchunks,
                        int num_cus, hipStream_t st) {
  LargeArgs L;
  L.a = a;
  L.inst = inst;
  L.n = n;
  L.nchunks = nchunks;
  L.ntb = (n + kLargeBlock - 1) / kLargeBlock;
  char* p = static_cast<char*>(scratch);
  auto take = [&](size_t bytes) {
    char* r = p;
    p += (bytes + 255) / 256 * 256;
    return r;
  };
  L.pos = reinterpret_cast<double*>(take(sizeof(double) * 2 * kS * n * 3));
  L.part = reinterpret_cast<double*>(take(sizeof(double) * (size_t)nchunks * kS * n * 3));
  L.rbuf = reinterpret_cast<double*>(take(sizeof(double) * 3 * n * kS));
  L.hist = reinterpret_cast<double*>(take(sizeof(double) * 3 * n * 2));
  L.arrive = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * L.ntb));
  L.flags = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * 9));
  L.ctl = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * 4));
  const int grid = kS * L.ntb * nchunks;
  int per_cu = 0;
  auto kern = a.exact ? large_kernel<true> : large_kernel<false>;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kLargeBlock, 0);
  if (e != hipSuccess) return e;
  if (grid > per_cu * num_cus) return hipErrorCooperativeLaunchTooLarge;
  // the step-end lanes must cover all 3n components
  if ((size_t)grid * kLargeBlock < (size_t)3 * n) return hipErrorInvalidConfiguration;
  void* args[] = {&L};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(kLargeBlock), args, 0, st);
}

}  // namespace irk

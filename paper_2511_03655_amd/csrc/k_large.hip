// IRKGL16 for one large gravitational system (more than 512 bodies, up to
// 8192, e.g. a 2048-body Plummer cluster): the whole GPU works on one system.
//
// One cooperative persistent launch per integration call.  The bodies are cut
// into groups of 8 targets; workgroup w owns groups w*gpw .. w*gpw+gpw-1, and
// in every wavefront lane (t, s) = 8 t + s stands for target t at stage s of
// the group at hand.  Per fixed-point iteration:
//  * force: for each owned group, the sources are split into 32 interleaved
//    chunks (b = c mod 32, ascending within a chunk) that the NCH wavefronts
//    of the workgroup take in turn from an LDS ticket counter (a fixed share
//    per wavefront let the oldest wavefront of each SIMD finish first and the
//    last one finish alone, at half the SIMD's FP64 issue rate).  Every
//    source is used by one wavefront only, so a wavefront stages its chunk's
//    stage positions in a region of LDS of its own, split into (x, y) and
//    (z, m) arrays [b][stage] so that the 8 stage entries it reads at once are
//    128 contiguous bytes; the force loop needs no workgroup barrier.  Chunk
//    partial sums go to per-chunk LDS slots and are added in chunk order, so
//    the result does not depend on which wavefront took which chunk;
//  * update, one component per wavefront (component d of group g by
//    wavefront 3 g + d): R_s = h b_s G g_s, stage values
//    Q_s = q + h (c_s v + sum_j eta_sj R_j) (eq. IRK_FP2) with the body's R_j
//    exchanged inside the wavefront, max-norm increments per component
//    (eq. Delta_n) by butterfly over the stage lanes, stopping rule
//    (eq. stopping); "not converged" / "non-finite" are OR-ed into the
//    workgroup's flag word.  The new stage positions go to the next position
//    buffer, and the next step's initial guess (eq. IRK_init2), formed after
//    a tentative compensated update (eq. qnvn2), to a third buffer;
//  * one grid barrier, whose last arriver publishes the OR of the
//    workgroups' flags with the release; every workgroup then either
//    iterates again from the new stage positions or commits the tentative
//    update and starts the next step from the guess buffer, so a step costs
//    exactly k grid barriers.
// The per-target state (q, v as two-double values, the stopping-rule history)
// lives in LDS, so the force loop runs without register spills.  Three
// position buffers rotate so that no buffer is written while it is read.
// With EXACT (reproducible mode) a single chunk is used and every sum runs in
// the reference order.
#include "device_common.h"
#include "pair_weight.h"

namespace irk {

constexpr int kLgT = 8;  // targets per group
constexpr int kLgMaxBodies = 8192;
constexpr int kBarSub = 16;  // first-level barrier counters

struct LargeArgs {
  LaunchArgs a;
  int32_t inst;     // instance id
  int32_t n;        // bodies
  int32_t ngroups;  // ceil(n / 8)
  int32_t gpw;      // groups per workgroup
  double* pos;      // [3 buffers][x, y, z, m][n bodies][8 stages]
  // barrier control words (see grid_barrier); the release word carries the
  // generation << 2 | flags (bit 0 not converged, bit 1 non-finite)
  unsigned* ctl;
};

template <int NCH, int TILE>
struct LargeCfg {
  static constexpr int kThreads = 64 * NCH;
  // source chunks per group and iteration, taken by the wavefronts in turn
  static constexpr int kChunks = NCH > 1 ? 32 : 1;
  static constexpr int kTile = TILE;                  // sources per LDS tile
  static constexpr int kMaxGroups = NCH > 1 ? 4 : 1;  // groups per workgroup
};

// Control words, one 128-byte line each: kBarSub first-level arrival
// counters, the top counter, the release word.
constexpr int kLine = 32;  // unsigned words per line
constexpr int kCtlWords = (kBarSub + 2) * kLine;
// Arrival increment: count in bits 0..15, "not converged" contributions in
// bits 16..23, "non-finite" contributions in bits 24..31 (at most 16
// arrivals per counter, so the fields never overflow).
__device__ __forceinline__ unsigned arrival_word(unsigned flags) {
  return 1u | ((flags & 1u) << 16) | ((flags & 2u) << 23);
}
__device__ __forceinline__ unsigned arrival_flags(unsigned total) {
  return ((total >> 16) & 0xFFu ? 1u : 0u) | ((total >> 24) ? 2u : 0u);
}

// Grid-wide barrier over co-resident workgroups (cooperative launch), two
// levels of arrival counters (16 first-level counters, then one top counter)
// so that no counter takes more than 16 arrivals, each counter on its own
// cache line.  A workgroup's flags (`*blk_flags`, OR-ed in LDS by its state
// wavefronts) ride on its arrival increment; the last arriver publishes the
// OR over all workgroups with the new generation in the release word, and the
// barrier returns it (through the LDS word `*res`, which no thread writes
// again before the next barrier).  `gen` counts this workgroup's barriers (identical in all
// threads).  Ordering: each arrival is preceded by a release fence; a
// workgroup that completes a counter acquires before resetting it and
// releases before passing on; waiters poll with plain atomic loads (no cache
// invalidation per poll) and acquire once.
__device__ __forceinline__ unsigned grid_barrier(unsigned* ctl, unsigned& gen, unsigned nblocks,
                                                 const unsigned* blk_flags, unsigned* res) {
  constexpr unsigned kMask = 0x3FFFFFFFu;
  unsigned* top = ctl + kBarSub * kLine;
  unsigned* rel = ctl + (kBarSub + 1) * kLine;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned j = blockIdx.x % kBarSub;
    const unsigned nsub = nblocks < (unsigned)kBarSub ? nblocks : (unsigned)kBarSub;
    const unsigned members = nblocks / kBarSub + (j < nblocks % kBarSub ? 1u : 0u);
    const unsigned mine = arrival_word(*blk_flags);
    unsigned* sub = ctl + j * kLine;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned old = __hip_atomic_fetch_add(sub, mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if ((old & 0xFFFFu) == members - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(sub, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned up = arrival_word(arrival_flags(old + mine));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned old2 = __hip_atomic_fetch_add(top, up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if ((old2 & 0xFFFFu) == nsub - 1) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned f = arrival_flags(old2 + up);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_store(rel, (((gen + 1) & kMask) << 2) | f, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    unsigned v;
    while (((v = __hip_atomic_load(rel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) >> 2) ==
           (gen & kMask))
      __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *res = v & 3u;
  }
  ++gen;
  __syncthreads();
  return *res;
}

// Maximum over the 8 stage lanes of a target; a non-finite operand is
// detected by the caller (finite() of its own increment), since fmax drops NaN.
__device__ __forceinline__ double lg_group_max(double x) {
#pragma unroll
  for (int m = 1; m < kS; m <<= 1) x = fmax(x, __shfl_xor(x, m, kS));
  return x;
}

__device__ __forceinline__ void lg_wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Own stage s of the initial guess (eq. IRK_init2) from increments Rp.
template <bool EXACT>
__device__ __forceinline__ double lg_guess(ConstTab T, int s, double q, double v,
                                           const double (&Rp)[kS], double h) {
  if constexpr (!EXACT) {  // folded matrix K, as initial_guess
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

// Weight m (r2 + eps2)^(-3/2) of one source (eps2 already in r2); fast form
// with one Halley step (mass_rinv3_halley).
template <bool EXACT>
__device__ __forceinline__ double lg_weight(double r2, double m) {
  if constexpr (EXACT)
    return pair_weight<EXACT>(r2, m);
  else
    return mass_rinv3_halley(r2, m);
}

// Squared distance in the reference order (EXACT) or with fused products.
template <bool EXACT>
__device__ __forceinline__ double lg_r2(double dx, double dy, double dz, double eps2) {
  if constexpr (EXACT) {
    double r2 = 0.0;
    r2 = r2 + dx * dx;
    r2 = r2 + dy * dy;
    r2 = r2 + dz * dz;
    return r2 + eps2;
  } else {
    return fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
  }
}

template <bool EXACT>
__device__ __forceinline__ void lg_acc(double w, double dx, double dy, double dz, double& acc0,
                                       double& acc1, double& acc2) {
  if constexpr (EXACT) {
    acc0 = acc0 + w * dx;
    acc1 = acc1 + w * dy;
    acc2 = acc2 + w * dz;
  } else {
    acc0 = fma(w, dx, acc0);
    acc1 = fma(w, dy, acc1);
    acc2 = fma(w, dz, acc2);
  }
}

// Accumulates the stage-s force on target `tgt` from one staged chunk of this
// wavefront's sources: local entries 0 .. cnt-1 hold global sources b0, b0 +
// NCH, b0 + 2 NCH, ... (ascending).  Two sources are evaluated as independent
// chains per loop trip (their contributions are still added in source order).
// SEL: replace the self distance (unsoftened forces); the self term then
// contributes w * 0 = 0.
template <bool EXACT, int NCH, bool SEL>
__device__ __forceinline__ void lg_force_chunk(const double2* __restrict__ sxy,
                                               const double2* __restrict__ szm, int cnt, int s,
                                               int b0, int tgt, double qx, double qy, double qz,
                                               double eps2, double& acc0, double& acc1,
                                               double& acc2) {
  int i = 0;
  for (; i + 1 < cnt; i += 2) {
    const double2 xa = sxy[i * kS + s], za = szm[i * kS + s];
    const double2 xb = sxy[(i + 1) * kS + s], zb = szm[(i + 1) * kS + s];
    const double dxa = xa.x - qx, dya = xa.y - qy, dza = za.x - qz;
    const double dxb = xb.x - qx, dyb = xb.y - qy, dzb = zb.x - qz;
    double r2a = lg_r2<EXACT>(dxa, dya, dza, eps2);
    double r2b = lg_r2<EXACT>(dxb, dyb, dzb, eps2);
    if constexpr (SEL) {
      r2a = (b0 + i * NCH == tgt) ? 1.0 : r2a;
      r2b = (b0 + (i + 1) * NCH == tgt) ? 1.0 : r2b;
    }
    const double wa = lg_weight<EXACT>(r2a, za.y);
    const double wb = lg_weight<EXACT>(r2b, zb.y);
    lg_acc<EXACT>(wa, dxa, dya, dza, acc0, acc1, acc2);
    lg_acc<EXACT>(wb, dxb, dyb, dzb, acc0, acc1, acc2);
  }
  if (i < cnt) {
    const double2 xa = sxy[i * kS + s], za = szm[i * kS + s];
    const double dxa = xa.x - qx, dya = xa.y - qy, dza = za.x - qz;
    double r2a = lg_r2<EXACT>(dxa, dya, dza, eps2);
    if constexpr (SEL) r2a = (b0 + i * NCH == tgt) ? 1.0 : r2a;
    lg_acc<EXACT>(lg_weight<EXACT>(r2a, za.y), dxa, dya, dza, acc0, acc1, acc2);
  }
}

// Store into a position buffer that the other workgroups read after the next
// grid barrier.  A relaxed atomic store at agent scope writes through this
// XCD's L2, so the L2 holds no dirty position lines when the barrier's release
// fence writes the L2 back (that write-back, once per workgroup and
// iteration, otherwise grows with every dirty line of the XCD).
__device__ __forceinline__ void pos_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-target state of a group in LDS (identical for the 8 stage lanes of a
// target, so stored once per target and component).
struct LgTargetState {
  double qh[kLgT][3], ql[kLgT][3], vh[kLgT][3], vl[kLgT][3];
  double mind[kLgT][3], prv[kLgT][3];  // stopping-rule history
};

template <bool EXACT, int NCH, int TILE>
__global__ __launch_bounds__(64 * NCH) void large_kernel(LargeArgs L) {
  constexpr int TB = LargeCfg<NCH, TILE>::kTile;
  constexpr int NT = LargeCfg<NCH, TILE>::kThreads;
  constexpr int GM = LargeCfg<NCH, TILE>::kMaxGroups;
  constexpr int CB = TB / NCH;       // sources per wavefront chunk
  constexpr int WENT = CB * kS / 64;  // chunk entries staged per lane
  static_assert(CB * kS % 64 == 0, "a chunk is a whole number of entries per lane");
  __shared__ double2 sxy[NCH][CB * kS];       // per wavefront: [source][stage] (x, y)
  __shared__ double2 szm[NCH][CB * kS];       // per wavefront: [source][stage] (z, m)
  constexpr int NCK = LargeCfg<NCH, TILE>::kChunks;
  __shared__ double part[NCK > 1 ? NCK : 1][3][64];  // chunk partial sums
  __shared__ unsigned tickets;                        // chunk tickets (never reset)
  __shared__ double tq[GM][3][64];            // current stage positions of the owned groups
  __shared__ double rt[GM][3][64];            // increments R of the owned groups
  __shared__ double gq[GM][3][64];            // tentative next-step initial guess
  __shared__ LgTargetState ts[GM];            // per-target state
  __shared__ double coef[kS][kS + 2];         // eta row, c, b per stage
  __shared__ unsigned blk_flags;  // this workgroup's flags for the next barrier
  __shared__ unsigned bar_res;    // flags returned by the last barrier

  const LaunchArgs& a = L.a;
  const ConstTab T = const_tab(a.tab);
  const InstDesc& dsc = a.desc[L.inst];
  const int n = L.n;
  const int dq = 3 * n;
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int t = lane >> 3, s = lane & 7;
  const unsigned nblocks = gridDim.x;
  const int gpw = L.gpw;
  const int g0 = blockIdx.x * gpw;
  // this wavefront's group, as state owner
  const int my_group = g0 + wave;
  const bool owner = wave < gpw && my_group < L.ngroups;
  const int my_tgt = my_group * kLgT + t;
  const bool mine = owner && my_tgt < n;

  const double* mass = a.params + dsc.mass_off;
  double* Sp = a.state + dsc.state_off;
  const double h = dsc.h;
  const double G = dsc.G;
  const double eps2 = dsc.eps * dsc.eps;
  const InstStat st0 = a.stat[L.inst];
  int64_t step = st0.steps_done;
  const int64_t target = launch_target(a, step, dsc.nsteps, st0.status);
  int64_t it_sum = st0.iterations, nonconv = st0.nonconv;
  int32_t maxk = st0.max_k;
  // barrier generation: continue from the release word left by the previous
  // launch (nobody can advance it before every workgroup has arrived once)
  unsigned gen = 0;
  if (tid == 0)
    gen = __hip_atomic_load(L.ctl + (kBarSub + 1) * kLine, __ATOMIC_RELAXED,
                            __HIP_MEMORY_SCOPE_AGENT) >> 2;

  for (int e = tid; e < kS * kS; e += NT) coef[e / kS][e % kS] = a.tab[kTabEta + e];
  if (tid < kS) {
    coef[tid][kS] = a.tab[kTabC + tid];
    coef[tid][kS + 1] = a.tab[kTabB + tid];
  }
  const size_t n8 = (size_t)n * kS;  // (body, stage) entries per component array
  const size_t bufsz = 4 * n8;       // doubles per position buffer
  double* pos = L.pos;
  int rbuf = 0;

  // ---- state and the first initial guess (into position buffer 0)
  if (owner) {
    LgTargetState& S = ts[wave];
#pragma unroll 1
    for (int d = 0; d < 3; ++d) {
      double q0 = 0.0, r0 = 0.0;
      if (mine && step < target) {
        const int c = my_tgt * 3 + d;
        const double qh = Sp[c], vh = Sp[2 * dq + c];
        S.qh[t][d] = qh;
        S.ql[t][d] = Sp[dq + c];
        S.vh[t][d] = vh;
        S.vl[t][d] = Sp[3 * dq + c];
        S.mind[t][d] = __builtin_inf();
        S.prv[t][d] = __builtin_inf();
        double Rp[kS];
#pragma unroll
        for (int j = 0; j < kS; ++j) Rp[j] = Sp[4 * dq + c * kS + j];
        r0 = Rp[s];
        q0 = lg_guess<EXACT>(T, s, qh, vh, Rp, h);
        pos_store(&pos[d * n8 + (size_t)my_tgt * kS + s], q0);
      }
      tq[wave][d][lane] = q0;
      rt[wave][d][lane] = r0;
    }
    // masses never change: written once per launch into all three buffers
    if (mine && step < target)
      for (int b = 0; b < 3; ++b)
        pos_store(&pos[b * bufsz + 3 * n8 + (size_t)my_tgt * kS + s], mass[my_tgt]);
  }
  if (tid == 0) {
    blk_flags = 0;
    tickets = 0;
  }
  unsigned tbase = 0;  // first ticket of the current group's chunks
  __threadfence();
  grid_barrier(L.ctl, gen, nblocks, &blk_flags, &bar_res);

  int k = 0;
  bool dead = false;
  while (step < target) {
    ++k;
    const int wb = (rbuf + 1) % 3, gb = (rbuf + 2) % 3;  // new stage values, next guess
    const double* P = pos + (size_t)rbuf * bufsz;
    if (tid == 0) blk_flags = 0;  // last read by thread 0 inside the previous barrier

    for (int g = 0; g < gpw; ++g) {
      const int grp = g0 + g;
      if (grp >= L.ngroups) break;  // uniform over the workgroup
      const int tgt = grp * kLgT + t;
      // ---- force on the group's targets.  The sources are split into NCK
      // interleaved chunks (b = c mod NCK, ascending within a chunk) that the
      // wavefronts take in turn from an LDS ticket counter, so the wavefronts
      // of a SIMD finish together instead of the oldest first; chunk c's
      // partial sums go to slot c and the update adds the slots in chunk
      // order, so the result does not depend on which wavefront took which
      // chunk.  A wavefront stages its chunk's sources in its own LDS region
      // (no other wavefront reads them: wavefront-level ordering suffices).
      // Lane (t, s) stages stage s of sources t, t + 8, ... of the chunk; the
      // next part is fetched into registers while the current one is used.
      double qx = 0.0, qy = 0.0, qz = 0.0;
      if (tgt < n) {
        qx = tq[g][0][lane];
        qy = tq[g][1][lane];
        qz = tq[g][2][lane];
      }
      // the update of the previous group has read its partial sums
      if constexpr (NCK > 1) {
        if (g > 0) __syncthreads();
      }
      double2* wxy = sxy[wave];
      double2* wzm = szm[wave];
      double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
      for (int taken = 0;; ++taken) {
        int c;
        if constexpr (NCK > 1) {
          unsigned tk = 0;
          if (lane == 0) tk = atomicAdd(&tickets, 1u);
          c = (int)(__builtin_amdgcn_readfirstlane(tk) - tbase);
        } else {
          c = taken;  // a single chunk, all sources in order
        }
        if (c >= NCK) break;
        acc0 = acc1 = acc2 = 0.0;
        const int nw = n > c ? (n - c + NCK - 1) / NCK : 0;  // sources of this chunk
        double pre[WENT][4];
#pragma unroll
        for (int r = 0; r < WENT; ++r) {
          const int i = t + 8 * r;
          if (i < nw) {
            const double* src = P + (size_t)(c + NCK * i) * kS + s;
#pragma unroll
            for (int q = 0; q < 4; ++q) pre[r][q] = src[q * n8];
          }
        }
        for (int j0 = 0; j0 < nw; j0 += CB) {
          const int cnt = min(CB, nw - j0);
          lg_wave_lds_sync();  // the previous part's reads are done
#pragma unroll
          for (int r = 0; r < WENT; ++r) {
            const int i = t + 8 * r;
            if (i < cnt) {
              wxy[i * kS + s] = make_double2(pre[r][0], pre[r][1]);
              wzm[i * kS + s] = make_double2(pre[r][2], pre[r][3]);
            }
          }
          lg_wave_lds_sync();
          const int j1 = j0 + CB;
          if (j1 < nw) {
#pragma unroll
            for (int r = 0; r < WENT; ++r) {
              const int i = j1 + t + 8 * r;
              if (i < nw) {
                const double* src = P + (size_t)(c + NCK * i) * kS + s;
#pragma unroll
                for (int q = 0; q < 4; ++q) pre[r][q] = src[q * n8];
              }
            }
          }
          if (tgt < n) {
            // with softening the self term needs no special case (w finite,
            // displacement 0); without it the self distance is replaced
            const int b0 = c + NCK * j0;
            if (eps2 > 0.0)
              lg_force_chunk<EXACT, NCK, false>(wxy, wzm, cnt, s, b0, tgt, qx, qy, qz, eps2,
                                                acc0, acc1, acc2);
            else
              lg_force_chunk<EXACT, NCK, true>(wxy, wzm, cnt, s, b0, tgt, qx, qy, qz, eps2,
                                               acc0, acc1, acc2);
          }
        }
        if constexpr (NCK > 1) {
          part[c][0][lane] = acc0;
          part[c][1][lane] = acc1;
          part[c][2][lane] = acc2;
        }
      }
      if constexpr (NCK > 1) {
        tbase += NCK + NCH;  // NCK chunks and one empty ticket per wavefront
        __syncthreads();
      }
      if (tgt < n) {
        // ---- update of group g: component d by wavefront (3 g + d) mod NCH
        const double hb = h * coef[s][kS + 1];
        const double cs = coef[s][kS];
        LgTargetState& S = ts[g];
        bool ok = true, bad = false, any = false;
#pragma unroll 1
        for (int d = 0; d < 3; ++d) {
          if ((3 * g + d) % NCH != wave) continue;  // uniform over the wavefront
          any = true;
          double gsum;
          if constexpr (NCH > 1) {
            gsum = part[0][d][lane];
#pragma unroll
            for (int c = 1; c < NCK; ++c) gsum += part[c][d][lane];
          } else {
            gsum = d == 0 ? acc0 : (d == 1 ? acc1 : acc2);
          }
          double Rn;
          if constexpr (EXACT)
            Rn = hb * (G * gsum);
          else
            Rn = (hb * G) * gsum;
          rt[g][d][lane] = Rn;
          lg_wave_lds_sync();
          double Rj[kS];
#pragma unroll
          for (int j = 0; j < kS; ++j) Rj[j] = rt[g][d][t * kS + j];
          const double qh = S.qh[t][d], vh = S.vh[t][d];
          double qn;
          if constexpr (EXACT) {
            double sm = 0.0;
#pragma unroll
            for (int j = 0; j < kS; ++j) sm = sm + coef[s][j] * Rj[j];
            qn = qh + h * (cs * vh + sm);
          } else {
            double acc = cs * vh;
#pragma unroll
            for (int j = 0; j < kS; ++j) acc = fma(coef[s][j], Rj[j], acc);
            qn = fma(h, acc, qh);
          }
          const double dd = fabs(qn - tq[g][d][lane]);
          bad |= !finite(dd);
          const double dmax = lg_group_max(dd);
          double mind = S.mind[t][d], prv = S.prv[t][d];
          ok &= stop_component(dmax, mind, prv);
          // tentative compensated update and the next step's initial guess
          double sv, sc;
          step_sums<EXACT>(row_tab(T), Rj, sv, sc);
          double vh2 = vh, vl2 = S.vl[t][d], qh2 = qh, ql2 = S.ql[t][d];
          dw_add(vh2, vl2, sv);
          dw_add(qh2, ql2, h * (vh2 - sc));
          const double qg = lg_guess<EXACT>(T, s, qh2, vh2, Rj, h);
          // all 8 stage lanes hold the same history; they store equal values
          S.mind[t][d] = mind;
          S.prv[t][d] = prv;
          tq[g][d][lane] = qn;
          gq[g][d][lane] = qg;
          // lanes (t, s) of the group are 64 consecutive entries of the
          // component array: one 512-byte store per wavefront
          pos_store(&pos[wb * bufsz + d * n8 + (size_t)tgt * kS + s], qn);
          pos_store(&pos[gb * bufsz + d * n8 + (size_t)tgt * kS + s], qg);
        }
        if (any) {
          const uint64_t notok = __ballot(!ok), badm = __ballot(bad);
          if (lane == 0 && (notok | badm))  // target 0 of a group always exists
            atomicOr(&blk_flags, (notok ? 1u : 0u) | (badm ? 2u : 0u));
        }
      }
    }
    const unsigned bits = grid_barrier(L.ctl, gen, nblocks, &blk_flags, &bar_res);
    if (bits & 2u) {
      dead = true;
      break;
    }
    const bool notok = (bits & 1u) != 0;
    const bool capped = notok && k >= a.max_iter;
    if (notok && !capped) {  // iterate again from the new stage positions (in tq)
      rbuf = wb;
      continue;
    }
    // ---- step accepted: commit the compensated update, outputs
    ++step;
    it_sum += k;
    nonconv += capped ? 1 : 0;
    maxk = k > maxk ? k : maxk;
    if (blockIdx.x == 0 && tid == 0 && dsc.iters_off >= 0)
      a.step_iters[dsc.iters_off + step - 1] = (uint8_t)k;
    k = 0;
    rbuf = gb;
    // component d of group g by wavefront 3 g + d (mod NCH), as in the update
    for (int u = wave; u < 3 * gpw; u += NCH) {
      const int g = u / 3, d = u % 3;
      const int tg = (g0 + g) * kLgT + t;
      if (g0 + g >= L.ngroups || tg >= n) continue;
      LgTargetState& S = ts[g];
      double Rj[kS];
#pragma unroll
      for (int j = 0; j < kS; ++j) Rj[j] = rt[g][d][t * kS + j];
      double sv, sc;
      step_sums<EXACT>(row_tab(T), Rj, sv, sc);
      double vh = S.vh[t][d], vl = S.vl[t][d], qh = S.qh[t][d], ql = S.ql[t][d];
      dw_add(vh, vl, sv);
      dw_add(qh, ql, h * (vh - sc));
      // every stage lane of the target computed the same values
      S.qh[t][d] = qh;
      S.ql[t][d] = ql;
      S.vh[t][d] = vh;
      S.vl[t][d] = vl;
      S.mind[t][d] = __builtin_inf();
      S.prv[t][d] = __builtin_inf();
      tq[g][d][lane] = gq[g][d][lane];
      if (s == 0 && step % dsc.stride == 0) {
        const int64_t fo = dsc.out_off + (step / dsc.stride) * dq + tg * 3;
        a.qout[fo + d] = qh;
        a.pout[fo + d] = mass[tg] * vh;
      }
    }
    __syncthreads();  // the new step's stage positions (tq) before any wavefront reads them
  }

  // ---- end of launch
  if (dead) {
    if (mine && s == 0) {
      const int64_t nf = target / dsc.stride;  // frames of this launch only
      for (int64_t f = step / dsc.stride + 1; f <= nf; ++f)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          a.qout[dsc.out_off + f * dq + my_tgt * 3 + d] = __builtin_nan("");
          a.pout[dsc.out_off + f * dq + my_tgt * 3 + d] = __builtin_nan("");
        }
    }
    if (blockIdx.x == 0 && tid == 0 && dsc.iters_off >= 0)
      a.step_iters[dsc.iters_off + step] = (uint8_t)k;
  } else if (mine && step > st0.steps_done) {
    const LgTargetState& S = ts[wave];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int c = my_tgt * 3 + d;
      if (s == 0) {
        Sp[c] = S.qh[t][d];
        Sp[dq + c] = S.ql[t][d];
        Sp[2 * dq + c] = S.vh[t][d];
        Sp[3 * dq + c] = S.vl[t][d];
      }
      Sp[4 * dq + c * kS + s] = rt[wave][d][lane];
    }
  }
  if (blockIdx.x == 0 && tid == 0) {
    InstStat st;
    st.steps_done = step;
    st.iterations = it_sum;
    st.nonconv = nonconv;
    st.max_k = maxk;
    st.status = dead ? kNonFinite : st0.status;
    a.stat[L.inst] = st;
  }
}

bool large_class_supported(int kind, int n, int d) {
  return kind == kGravity && d == 3 && n > 1 && n <= kLgMaxBodies;
}

// Device scratch for a system of n bodies: the control words (at a fixed
// offset, zeroed once when the buffer is allocated: every barrier leaves its
// counters at zero and the release word carries over between launches), then
// three position buffers.
constexpr size_t kCtlBytes = 4096;
static_assert(sizeof(unsigned) * kCtlWords <= kCtlBytes, "control block");
size_t large_scratch_bytes(int n, int /*nchunks*/) {
  return kCtlBytes + sizeof(double) * (size_t)3 * n * kS * 4;
}
size_t large_control_bytes() { return kCtlBytes; }

// Source chunks (wavefronts per workgroup): 16, or 1 in reproducible mode.
int large_chunks(int /*n*/, bool exact, int /*num_cus*/) { return exact ? 1 : 16; }

template <bool EXACT, int NCH, int TILE>
static hipError_t launch_large_t(LargeArgs& L, int num_cus, hipStream_t st) {
  auto kern = large_kernel<EXACT, NCH, TILE>;
  constexpr int NT = LargeCfg<NCH, TILE>::kThreads;
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, NT, 0);
  if (e != hipSuccess) return e;
  if (per_cu < 1) return hipErrorCooperativeLaunchTooLarge;
  const int cap = per_cu * num_cus;
  // fewest groups per workgroup such that the grid is co-resident
  int gpw = (L.ngroups + cap - 1) / cap;
  if (gpw < 1) gpw = 1;
  if (gpw > LargeCfg<NCH, TILE>::kMaxGroups) return hipErrorCooperativeLaunchTooLarge;
  L.gpw = gpw;
  const int grid = (L.ngroups + gpw - 1) / gpw;
  void* args[] = {&L};
  return hipLaunchCooperativeKernel((const void*)kern, dim3(grid), dim3(NT), args, 0, st);
}

hipError_t launch_large(const LaunchArgs& a, int inst, int n, void* scratch, int /*nchunks*/,
                        int num_cus, hipStream_t st, int tile) {
  if (n < 2 || n > kLgMaxBodies) return hipErrorInvalidValue;
  LargeArgs L;
  L.a = a;
  L.inst = inst;
  L.n = n;
  L.ngroups = (n + kLgT - 1) / kLgT;
  L.gpw = 1;
  char* p = static_cast<char*>(scratch);
  L.ctl = reinterpret_cast<unsigned*>(p);
  L.pos = reinterpret_cast<double*>(p + kCtlBytes);
  if (a.exact) return launch_large_t<true, 1, 64>(L, num_cus, st);
  if (tile == 128) return launch_large_t<false, 16, 128>(L, num_cus, st);
  return launch_large_t<false, 16, 256>(L, num_cus, st);
}

}  // namespace irk

/*
 * Plain FP64 oracle for the explicit symplectic baselines of section 4:
 * symmetric compositions of Strang steps (eq. Strang, eq. comp_method) run in
 * their ABA form (eq. high_order_splitting) with the exact flows of eq.
 * flowAB for a separable Hamiltonian (q' = v drift, v' = g(q) kick):
 *
 *   for j = 1..s:  q <- q (+) fl(fl(a_j h) v.hi);
 *                  v <- v (+) fl(fl(b_j h) g(q.hi, t_j)),  t_j = fl(fl((n-1) h) + fl(c_j h))
 *   then           q <- q (+) fl(fl(a_{s+1} h) v.hi)
 *
 * with q, v kept as two-double values and x (+) d the same compensated
 * addition as the IRKGL16 oracle (the paper runs its splitting baselines with
 * compensated summation, section 5.2).  c_j = a_1 + ... + a_j is the time
 * fraction reached by the drifts before the j-th kick.  Methods: Strang
 * (s = 1) and SUZ90 (Suzuki 1990, order 4, s = 5); coefficients from
 * tableau.h.
 *
 * TEST INFRASTRUCTURE ONLY: shares nothing with the GPU library; only the
 * test-suite, the smoke check and the benchmark's CPU-baseline leg load it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tableau.h"

typedef struct {
  int32_t kind, n, d;
  const double *mass;
  const double *coupling;
  double G, eps, beta;
} split_problem;

typedef struct {
  int64_t steps_done;
  int64_t iterations;
  int32_t max_k;
  int32_t nonconverged;
  int32_t status;
} split_stats;

enum { SPLIT_STRANG = 1, SPLIT_SUZ90 = 2 };
enum { SPL_OK = 0, SPL_EINVAL = -1, SPL_ENOMEM = -2, SPL_ENONFINITE = -4 };

/* from irkgl16_oracle.c */
void orc_force_t(const split_problem *p, const double *Q, double *G, double t);
void orc_dw_add(double *hi, double *lo, double delta);

static double split_mass(const split_problem *p, int body) {
  if (p->kind == 1) return p->mass[body];                 /* gravity */
  if (p->kind == 2) return p->mass ? p->mass[body] : 1.0; /* chain */
  return 1.0;
}

/* (a, b, c, s) of a method, or 0. */
static int split_tables(int method, const double **a, const double **b, const double **c) {
  switch (method) {
  case SPLIT_STRANG: *a = ORC_STRANG_A; *b = ORC_STRANG_B; *c = ORC_STRANG_C; return 1;
  case SPLIT_SUZ90: *a = ORC_SUZ90_A; *b = ORC_SUZ90_B; *c = ORC_SUZ90_C; return 5;
  }
  return 0;
}

/*
 * One instance of a second-order problem (the kinds of irkgl16_oracle.c).
 * q0, p0: Dq values; frames [frame][Dq] of q.hi and p = m v.hi every stride
 * steps (frame 0: initial state).  Returns 0, SPL_EINVAL or SPL_ENONFINITE
 * (the instance stops at the first non-finite state; later frames NaN).
 */
int orc_split_integrate(const split_problem *p, int32_t method, const double *q0,
                        const double *p0, double h, int64_t nsteps, int64_t stride,
                        double *q_out, double *p_out, split_stats *st) {
  const double *A, *B, *Cf;
  const int s = split_tables(method, &A, &B, &Cf);
  if (!s || p->n < 1 || p->d < 1 || !isfinite(h) || nsteps < 0 || stride < 1 ||
      nsteps % stride)
    return SPL_EINVAL;
  const int Dq = p->n * p->d;
  double *buf = (double *)calloc((size_t)Dq * 5, sizeof(double));
  if (!buf) return SPL_ENOMEM;
  double *qh = buf, *ql = qh + Dq, *vh = ql + Dq, *vl = vh + Dq, *G = vl + Dq;
  double ah[6], bh[5], ch[5];
  for (int j = 0; j <= s; ++j) ah[j] = h * A[j];
  for (int j = 0; j < s; ++j) {
    bh[j] = h * B[j];
    ch[j] = Cf[j] * h;
  }
  for (int l = 0; l < Dq; ++l) {
    qh[l] = q0[l];
    vh[l] = p0[l] / split_mass(p, l / p->d);
    q_out[l] = qh[l];
    p_out[l] = split_mass(p, l / p->d) * vh[l];
  }
  split_stats loc = {0, 0, 0, 0, SPL_OK};
  int dead = 0;
  for (int64_t n = 1; n <= nsteps; ++n) {
    if (!dead) {
      const double t_prev = (double)(n - 1) * h;
      for (int j = 0; j < s; ++j) {
        for (int l = 0; l < Dq; ++l) orc_dw_add(qh + l, ql + l, ah[j] * vh[l]);
        orc_force_t(p, qh, G, t_prev + ch[j]);
        for (int l = 0; l < Dq; ++l) orc_dw_add(vh + l, vl + l, bh[j] * G[l]);
      }
      for (int l = 0; l < Dq; ++l) orc_dw_add(qh + l, ql + l, ah[s] * vh[l]);
      for (int l = 0; l < Dq; ++l)
        if (!isfinite(qh[l]) || !isfinite(vh[l])) dead = 1;
      if (dead)
        loc.status = SPL_ENONFINITE;
      else
        loc.steps_done = n;
    }
    if (n % stride == 0) {
      const int64_t f = n / stride;
      for (int l = 0; l < Dq; ++l) {
        q_out[f * Dq + l] = dead ? NAN : qh[l];
        p_out[f * Dq + l] = dead ? NAN : split_mass(p, l / p->d) * vh[l];
      }
    }
  }
  if (st) *st = loc;
  free(buf);
  return loc.status;
}

/* Many instances (OpenMP), packed as the GPU library packs them. */
int orc_split_integrate_batch(int32_t n_inst, int32_t method, const split_problem *probs,
                              const double *q0, const double *p0, const double *h,
                              const int64_t *nsteps, const int64_t *stride, double *q_out,
                              double *p_out, int32_t *status) {
  int64_t *in_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  int64_t *out_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  if (!in_off || !out_off) {
    free(in_off);
    free(out_off);
    return SPL_ENOMEM;
  }
  in_off[0] = out_off[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    const int64_t Dq = (int64_t)probs[i].n * probs[i].d;
    if (stride[i] < 1 || nsteps[i] < 0 || nsteps[i] % stride[i]) {
      free(in_off);
      free(out_off);
      return SPL_EINVAL;
    }
    in_off[i + 1] = in_off[i] + Dq;
    out_off[i + 1] = out_off[i] + Dq * (nsteps[i] / stride[i] + 1);
  }
  int worst = SPL_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_inst; ++i) {
    int rc = orc_split_integrate(probs + i, method, q0 + in_off[i], p0 + in_off[i], h[i],
                                 nsteps[i], stride[i], q_out + out_off[i], p_out + out_off[i],
                                 NULL);
    if (status) status[i] = rc;
    if (rc < 0) {
#pragma omp critical
      if (rc < worst) worst = rc;
    }
  }
  free(in_off);
  free(out_off);
  return worst;
}

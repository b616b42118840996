/*
 * Plain FP64 oracle for fixed-step IRKGL16 in the floating-point-symplectic
 * second-order (eta) formulation (and, with orc_integrate_s, for the s-stage
 * members s = 2, 4, 6 of the same family: the same steps with s in place of 8).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct CPU
 * reference that the GPU library is checked against.  It shares no code,
 * header, table or helper with the GPU library; only the test-suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * (strict IEEE binary64: no contraction into fma, no reassociation).
 *
 * What one step computes (second-order problem q'' = g(q, t), v = q'; eq.
 * ivp2, the force may depend on time):
 *   initial guess (section 2.5, eq. IRK_init2; eq. Pol0 for nu):
 *       V0_i = v + sum_j nu_ij R_prev_j
 *       L0_j = hb_j V0_j
 *       Q_i  = q + sum_j mu_ij L0_j
 *   fixed-point iteration k = 1, 2, ... (eq. IRK_FP2, eqs. Gi/Qi2):
 *       G_i  = g(Q_i, t_i),  t_i = fl(fl((n-1) h) + fl(c_i h))  for step n
 *              (the stage times t_{n-1} + c_i h of eq. IRK_FP, with t_0 = 0)
 *       R_i  = hb_i G_i                         (hb_i = fl(h b_i))
 *       Qn_i = q + h (c_i v + sum_j eta_ij R_j)
 *       Delta^l = max_i |Qn_i^l - Q_i^l|        (eq. Delta_n)
 *       Q = Qn; stop when, for every position component l, Delta^l == 0 or
 *       min(Delta^l[1..k-2]) <= min(Delta^l[k-1], Delta^l[k])  (eq. stopping)
 *   update (eq. qnvn2) with double-word state (section 5, compensated
 *   summation with a two-double state):
 *       S_v = sum_i R_i,  S_c = sum_i c_i R_i
 *       v <- v (+) S_v;   q <- q (+) h (v.hi - S_c);   R_prev <- R
 *   where x (+) d is: (s,e) = TwoSum(x.hi, d); t = e + x.lo;
 *   (x.hi, x.lo) = Fast2Sum(s, t).
 * Stage values only read the hi parts of q and v.  The R that drives the
 * update is the last one computed (from the previous iterate), so a step costs
 * exactly 8k force evaluations.  All sums run in ascending index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "tableau.h"

#define S 8

enum {
  ORC_KEPLER = 0,
  ORC_GRAVITY = 1,
  ORC_CHAIN = 2,
  /* problems used only by oracle pins */
  ORC_HARMONIC = 10, /* g = -G q               */
  ORC_CONST = 11,    /* g = G (every component) */
  ORC_HENON = 12,    /* Henon-Heiles, Dq = 2    */
  ORC_HENON_T = 13,  /* section 3.3's non-autonomous Henon-Heiles, Dq = 2:
                        lambda = G, xi = beta                            */
  ORC_DRIVEN = 14,   /* g = G cos(t) (every component)                   */
};

enum {
  ORC_FLAG_NO_COMPENSATION = 1, /* negative control: plain state update   */
  ORC_FLAG_NAIVE_ETA = 2,       /* negative control: eta without completion */
  ORC_FLAG_NO_EXTRAPOLATION = 4 /* initial guess with R_prev = 0 every step */
};

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ENONFINITE = -4, ORC_ENOCONV = 1 };

typedef struct {
  int32_t kind, n, d;
  const double *mass;     /* GRAVITY: n masses; CHAIN: n site masses or NULL */
  const double *coupling; /* CHAIN: n+1 bond stiffnesses or NULL             */
  double G, eps, beta;
} orc_problem;

typedef struct {
  int64_t steps_done;
  int64_t iterations;       /* sum of k over steps */
  int32_t max_k;
  int32_t nonconverged;     /* steps that hit max_iter */
  int32_t status;
} orc_stats;

/* ---------------- forces g(Q) ---------------- */

/* Gravitational systems of at least this many bodies spread their targets
 * over threads when the caller is not already parallel (one large system).
 * Each target's sum still runs over b in ascending order on one thread, so
 * the result is the same for any thread count. */
#define ORC_PAR_MIN_BODIES 256

static int orc_serial_caller(void) {
#ifdef _OPENMP
  return !omp_in_parallel();
#else
  return 0;
#endif
}

/* Thread count of the oracle's parallel loops for the calling thread (n <= 0:
 * back to the count in effect before the first call, i.e. OMP_NUM_THREADS or
 * the OpenMP default). */
void orc_set_threads(int n) {
#ifdef _OPENMP
  static int initial = 0;
  if (initial == 0) initial = omp_get_max_threads();
  omp_set_num_threads(n > 0 ? n : initial);
#else
  (void)n;
#endif
}

static double mass_of(const orc_problem *p, int body) {
  if (p->kind == ORC_GRAVITY) return p->mass[body];
  if (p->kind == ORC_CHAIN) return p->mass ? p->mass[body] : 1.0;
  return 1.0;
}

static double dV(double s, double beta) { return s + beta * (s * s * s); }

/* Softened Newtonian acceleration of body a (eq. Ham2): sources b != a in
 * ascending order. */
static void gravity_target(const orc_problem *p, const double *Q, double *G, int a) {
  const int n = p->n, d = p->d;
  const double eps2 = p->eps * p->eps;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < n; ++b) {
    if (b == a) continue;
    double dx[3], r2 = 0.0;
    for (int k = 0; k < d; ++k) {
      dx[k] = Q[b * d + k] - Q[a * d + k];
      r2 += dx[k] * dx[k];
    }
    r2 += eps2;
    double w = p->mass[b] / (r2 * sqrt(r2));
    for (int k = 0; k < d; ++k) acc[k] += w * dx[k];
  }
  for (int k = 0; k < d; ++k) G[a * d + k] = p->G * acc[k];
}

/* g(Q, t); the autonomous kinds ignore t. */
void orc_force_t(const orc_problem *p, const double *Q, double *G, double t) {
  const int n = p->n, d = p->d, Dq = n * d;
  switch (p->kind) {
  case ORC_KEPLER: {
    double r2 = 0.0;
    for (int k = 0; k < Dq; ++k) r2 += Q[k] * Q[k];
    double r3 = r2 * sqrt(r2);
    for (int k = 0; k < Dq; ++k) G[k] = -p->G * Q[k] / r3;
    break;
  }
  case ORC_GRAVITY: {
    /* a small system stays out of the OpenMP runtime altogether: even a
     * parallel region that runs on one thread costs more than its force */
    if (n >= ORC_PAR_MIN_BODIES && orc_serial_caller()) {
#pragma omp parallel for schedule(static)
      for (int a = 0; a < n; ++a) gravity_target(p, Q, G, a);
    } else {
      for (int a = 0; a < n; ++a) gravity_target(p, Q, G, a);
    }
    break;
  }
  case ORC_CHAIN: {
    for (int i = 0; i < n; ++i) {
      double ql = (i > 0) ? Q[i - 1] : 0.0;
      double qr = (i < n - 1) ? Q[i + 1] : 0.0;
      double kl = p->coupling ? p->coupling[i] : 1.0;
      double kr = p->coupling ? p->coupling[i + 1] : 1.0;
      double F = kr * dV(qr - Q[i], p->beta) - kl * dV(Q[i] - ql, p->beta);
      G[i] = F / mass_of(p, i);
    }
    break;
  }
  case ORC_HARMONIC:
    for (int k = 0; k < Dq; ++k) G[k] = -p->G * Q[k];
    break;
  case ORC_CONST:
    for (int k = 0; k < Dq; ++k) G[k] = p->G;
    break;
  case ORC_HENON:
    G[0] = -Q[0] - 2.0 * Q[0] * Q[1];
    G[1] = -Q[1] - (Q[0] * Q[0] - Q[1] * Q[1]);
    break;
  case ORC_HENON_T: {
    /* dp1/dt = -q1 - 2 a q1 q2, dp2/dt = -q2 - a (q1^2 - q2^2), a = lambda + xi sin t */
    double a = p->G + p->beta * sin(t);
    G[0] = -Q[0] - 2.0 * a * Q[0] * Q[1];
    G[1] = -Q[1] - a * (Q[0] * Q[0] - Q[1] * Q[1]);
    break;
  }
  case ORC_DRIVEN:
    for (int k = 0; k < Dq; ++k) G[k] = p->G * cos(t);
    break;
  }
}

void orc_force(const orc_problem *p, const double *Q, double *G) { orc_force_t(p, Q, G, 0.0); }

/* Hamiltonian H(q, p) of each problem (for energy-error pins). */
double orc_energy(const orc_problem *pr, const double *q, const double *p) {
  const int n = pr->n, d = pr->d, Dq = n * d;
  double T = 0.0, U = 0.0;
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < d; ++k) T += p[a * d + k] * p[a * d + k] / (2.0 * mass_of(pr, a));
  switch (pr->kind) {
  case ORC_KEPLER: {
    double r2 = 0.0;
    for (int k = 0; k < Dq; ++k) r2 += q[k] * q[k];
    U = -pr->G / sqrt(r2);
    break;
  }
  case ORC_GRAVITY: {
    double eps2 = pr->eps * pr->eps;
    for (int a = 0; a < n; ++a)
      for (int b = a + 1; b < n; ++b) {
        double r2 = 0.0;
        for (int k = 0; k < d; ++k) {
          double dx = q[b * d + k] - q[a * d + k];
          r2 += dx * dx;
        }
        U -= pr->G * pr->mass[a] * pr->mass[b] / sqrt(r2 + eps2);
      }
    break;
  }
  case ORC_CHAIN:
    for (int i = 0; i <= n; ++i) {
      double ql = (i > 0) ? q[i - 1] : 0.0;
      double qr = (i < n) ? q[i] : 0.0;
      double s = qr - ql, k = pr->coupling ? pr->coupling[i] : 1.0;
      U += k * (0.5 * s * s + 0.25 * pr->beta * s * s * s * s);
    }
    break;
  case ORC_HARMONIC:
    for (int k = 0; k < Dq; ++k) U += 0.5 * pr->G * q[k] * q[k];
    break;
  case ORC_CONST:
    for (int k = 0; k < Dq; ++k) U -= pr->G * q[k];
    break;
  case ORC_HENON:
    U = 0.5 * (q[0] * q[0] + q[1] * q[1]) + q[0] * q[0] * q[1] - q[1] * q[1] * q[1] / 3.0;
    break;
  case ORC_HENON_T: /* at t = 0: a = lambda */
    U = 0.5 * (q[0] * q[0] + q[1] * q[1]) + pr->G * (q[0] * q[0] * q[1] - q[1] * q[1] * q[1] / 3.0);
    break;
  case ORC_DRIVEN: /* at t = 0 */
    for (int k = 0; k < Dq; ++k) U -= pr->G * q[k];
    break;
  }
  return T + U;
}

/* ---------------- double-word helpers ---------------- */

/* x (+) delta: (s,e) = TwoSum(hi, delta) [Knuth]; t = e + lo;
 * (hi, lo) = Fast2Sum(s, t) [Dekker]. */
static void dw_add(double *hi, double *lo, double delta) {
  double s = *hi + delta;
  double bv = s - *hi;
  double e = (*hi - (s - bv)) + (delta - bv);
  double t = e + *lo;
  double h2 = s + t;
  *lo = t - (h2 - s);
  *hi = h2;
}

void orc_dw_add(double *hi, double *lo, double delta) { dw_add(hi, lo, delta); }

/* The stopping rule (eq. stopping) for one component.  `mind` holds
 * min(Delta[1..k-2]) and `prev` holds Delta[k-1] (both +inf initially).
 * Returns 1 if this component allows stopping, and advances the history. */
static int stop_component(double delta, double *mind, double *prev) {
  double m = (*prev < delta) ? *prev : delta;
  int ok = (delta == 0.0) || (*mind <= m);
  if (*prev < *mind) *mind = *prev;
  *prev = delta;
  return ok;
}

int orc_stop_component(double delta, double *mind, double *prev) {
  return stop_component(delta, mind, prev);
}

/* ---------------- one instance ---------------- */

static int valid_problem(const orc_problem *p) {
  if (p->n < 1 || p->d < 1 || p->d > 3) return 0;
  switch (p->kind) {
  case ORC_KEPLER: return p->n == 1;
  case ORC_GRAVITY:
    if (!p->mass) return 0;
    for (int a = 0; a < p->n; ++a)
      if (!(p->mass[a] > 0.0)) return 0;
    return 1;
  case ORC_CHAIN: return p->d == 1;
  case ORC_HARMONIC: case ORC_CONST: return 1;
  case ORC_HENON: case ORC_HENON_T: return p->n * p->d == 2;
  case ORC_DRIVEN: return 1;
  }
  return 0;
}

/* The coefficient tables of one member of the family: s stages, c and b of
 * length s, eta, mu, nu row-major s x s (row = stage formed). */
typedef struct {
  int s;
  const double *c, *b, *eta, *mu, *nu;
} orc_tab;

/* One instance with the tables of T (the steps listed at the top of this
 * file, with s in place of 8).  Arguments as orc_integrate. */
static int integrate_core(const orc_problem *p, const orc_tab *T, const double *q0,
                          const double *p0, double h, int64_t nsteps, int64_t stride,
                          int32_t max_iter, int32_t flags, double *q_out, double *p_out,
                          int32_t *iters, double *delta1, orc_stats *st) {
  if (!valid_problem(p) || !(isfinite(h)) || nsteps < 0 || stride < 1 || nsteps % stride ||
      max_iter < 1)
    return ORC_EINVAL;
  const int s = T->s;
  const int Dq = p->n * p->d;
  double *buf = (double *)calloc((size_t)Dq * (6 + 6 * s), sizeof(double));
  if (!buf) return ORC_ENOMEM;
  double *qh = buf, *ql = qh + Dq, *vh = ql + Dq, *vl = vh + Dq, *mind = vl + Dq,
         *prev = mind + Dq;
  double *Q = prev + Dq, *Qn = Q + s * Dq, *G = Qn + s * Dq, *R = G + s * Dq,
         *Rp = R + s * Dq, *V0 = Rp + s * Dq;
  const double *eta = T->eta, *mu = T->mu, *nu = T->nu, *cc = T->c;
  double hb[S];
  for (int i = 0; i < s; ++i) hb[i] = h * T->b[i];
  for (int l = 0; l < Dq; ++l) {
    qh[l] = q0[l];
    vh[l] = p0[l] / mass_of(p, l / p->d);
  }
  orc_stats loc = {0, 0, 0, 0, ORC_OK};
  int64_t frame = 0;
  for (int l = 0; l < Dq; ++l) {
    q_out[l] = qh[l];
    p_out[l] = mass_of(p, l / p->d) * vh[l];
  }
  int dead = 0;
  for (int64_t n = 1; n <= nsteps; ++n) {
    if (!dead) {
      if (flags & ORC_FLAG_NO_EXTRAPOLATION) memset(Rp, 0, sizeof(double) * s * Dq);
      /* initial guess */
      for (int i = 0; i < s; ++i)
        for (int l = 0; l < Dq; ++l) {
          double sum = 0.0;
          for (int j = 0; j < s; ++j) sum += nu[i * s + j] * Rp[j * Dq + l];
          V0[i * Dq + l] = vh[l] + sum;
        }
      for (int i = 0; i < s; ++i)
        for (int l = 0; l < Dq; ++l) {
          double sum = 0.0;
          for (int j = 0; j < s; ++j) sum += mu[i * s + j] * (hb[j] * V0[j * Dq + l]);
          Q[i * Dq + l] = qh[l] + sum;
        }
      for (int l = 0; l < Dq; ++l) mind[l] = prev[l] = INFINITY;
      /* fixed-point iteration */
      int k = 0, conv = 0;
      while (!conv && k < max_iter) {
        ++k;
        const double t_prev = (double)(n - 1) * h;
        for (int i = 0; i < s; ++i) orc_force_t(p, Q + i * Dq, G + i * Dq, t_prev + cc[i] * h);
        for (int i = 0; i < s; ++i)
          for (int l = 0; l < Dq; ++l) R[i * Dq + l] = hb[i] * G[i * Dq + l];
        for (int i = 0; i < s; ++i)
          for (int l = 0; l < Dq; ++l) {
            double sum = 0.0;
            for (int j = 0; j < s; ++j) sum += eta[i * s + j] * R[j * Dq + l];
            Qn[i * Dq + l] = qh[l] + h * (cc[i] * vh[l] + sum);
          }
        conv = 1;
        double dmax = 0.0;
        for (int l = 0; l < Dq; ++l) {
          double dl = 0.0;
          for (int i = 0; i < s; ++i) {
            double a = fabs(Qn[i * Dq + l] - Q[i * Dq + l]);
            if (isnan(a) || a > dl) dl = a; /* a NaN, once seen, is kept */
          }
          if (!isfinite(dl)) dead = 1;
          if (dl > dmax) dmax = dl;
          if (!stop_component(dl, mind + l, prev + l)) conv = 0;
        }
        if (k == 1 && delta1) delta1[n - 1] = dmax;
        memcpy(Q, Qn, sizeof(double) * s * Dq);
        if (dead) break;
      }
      if (!dead) {
        if (!conv) ++loc.nonconverged;
        loc.iterations += k;
        if (k > loc.max_k) loc.max_k = k;
        if (iters) iters[n - 1] = k;
        /* update with compensated summation */
        for (int l = 0; l < Dq; ++l) {
          double sv = 0.0, sc = 0.0;
          for (int i = 0; i < s; ++i) sv += R[i * Dq + l];
          for (int i = 0; i < s; ++i) sc += cc[i] * R[i * Dq + l];
          if (flags & ORC_FLAG_NO_COMPENSATION) {
            vh[l] += sv;
            qh[l] += h * (vh[l] - sc);
          } else {
            dw_add(vh + l, vl + l, sv);
            dw_add(qh + l, ql + l, h * (vh[l] - sc));
          }
        }
        memcpy(Rp, R, sizeof(double) * s * Dq);
        loc.steps_done = n;
      } else {
        loc.status = ORC_ENONFINITE;
        if (iters) iters[n - 1] = k;
      }
    } else if (iters) {
      iters[n - 1] = 0;
    }
    if (n % stride == 0) {
      ++frame;
      for (int l = 0; l < Dq; ++l) {
        q_out[frame * Dq + l] = dead ? NAN : qh[l];
        p_out[frame * Dq + l] = dead ? NAN : mass_of(p, l / p->d) * vh[l];
      }
    }
  }
  if (loc.status == ORC_OK && loc.nonconverged) loc.status = ORC_ENOCONV;
  if (st) *st = loc;
  free(buf);
  return loc.status;
}

/* Tables of the s-stage member (s = 2, 4, 6, 8), or 0 for another s. */
int orc_stage_tables(int s, orc_tab *T) {
  T->s = s;
  switch (s) {
  case 2: T->c = ORC_S2_C; T->b = ORC_S2_B; T->eta = &ORC_S2_ETA[0][0]; T->mu = &ORC_S2_MU[0][0]; T->nu = &ORC_S2_NU[0][0]; return 1;
  case 4: T->c = ORC_S4_C; T->b = ORC_S4_B; T->eta = &ORC_S4_ETA[0][0]; T->mu = &ORC_S4_MU[0][0]; T->nu = &ORC_S4_NU[0][0]; return 1;
  case 6: T->c = ORC_S6_C; T->b = ORC_S6_B; T->eta = &ORC_S6_ETA[0][0]; T->mu = &ORC_S6_MU[0][0]; T->nu = &ORC_S6_NU[0][0]; return 1;
  case 8: T->c = ORC_C; T->b = ORC_B; T->eta = &ORC_ETA[0][0]; T->mu = &ORC_MU[0][0]; T->nu = &ORC_NU[0][0]; return 1;
  }
  return 0;
}

/*
 * Integrate one instance with IRKGL16 (s = 8).  q0, p0: Dq values.  Frames
 * f = 0..nsteps/stride (state after f*stride steps; frame 0 is the initial
 * state) are written to q_out/p_out as [frame][Dq] with p = m * v.hi.  iters
 * (nullable): k of each step.  delta1 (nullable): max over components of
 * Delta^[1] of each step.  After a non-finite Delta the instance stops and its
 * remaining frames are NaN.  flags: the negative controls above.
 */
int orc_integrate(const orc_problem *p, const double *q0, const double *p0, double h,
                  int64_t nsteps, int64_t stride, int32_t max_iter, int32_t flags,
                  double *q_out, double *p_out, int32_t *iters, double *delta1,
                  orc_stats *st) {
  double eta[S][S];
  for (int i = 0; i < S; ++i)
    for (int j = 0; j < S; ++j)
      eta[i][j] = ((flags & ORC_FLAG_NAIVE_ETA) && j > i) ? ORC_ETA_NAIVE[i][j] : ORC_ETA[i][j];
  orc_tab T;
  orc_stage_tables(S, &T);
  T.eta = &eta[0][0];
  return integrate_core(p, &T, q0, p0, h, nsteps, stride, max_iter, flags, q_out, p_out, iters,
                        delta1, st);
}

/* The same with the s-stage member of the family (s = 2, 4, 6, 8; the
 * method of order 2s), no negative-control flags. */
int orc_integrate_s(const orc_problem *p, int32_t s, const double *q0, const double *p0,
                    double h, int64_t nsteps, int64_t stride, int32_t max_iter, double *q_out,
                    double *p_out, int32_t *iters, orc_stats *st) {
  orc_tab T;
  if (!orc_stage_tables(s, &T)) return ORC_EINVAL;
  return integrate_core(p, &T, q0, p0, h, nsteps, stride, max_iter, 0, q_out, p_out, iters,
                        NULL, st);
}

/*
 * Many instances (OpenMP across instances).  Packing: instance i has
 * Dq_i = n_i d_i values in q0/p0 (concatenated in order) and
 * F_i = nsteps_i / stride_i + 1 frames of Dq_i values in q_out/p_out.
 * iters_total[i] = sum of k; status[i] = per-instance code.
 */
int orc_integrate_batch(int32_t n_inst, const orc_problem *probs, const double *q0,
                        const double *p0, const double *h, const int64_t *nsteps,
                        const int64_t *stride, int32_t max_iter, int32_t flags, double *q_out,
                        double *p_out, int64_t *iters_total, int32_t *status) {
  int64_t *in_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  int64_t *out_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  if (!in_off || !out_off) {
    free(in_off);
    free(out_off);
    return ORC_ENOMEM;
  }
  in_off[0] = out_off[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    int64_t Dq = (int64_t)probs[i].n * probs[i].d;
    if (stride[i] < 1 || nsteps[i] < 0 || nsteps[i] % stride[i]) {
      free(in_off);
      free(out_off);
      return ORC_EINVAL;
    }
    in_off[i + 1] = in_off[i] + Dq;
    out_off[i + 1] = out_off[i] + Dq * (nsteps[i] / stride[i] + 1);
  }
  int worst = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_inst; ++i) {
    orc_stats st;
    int rc = orc_integrate(probs + i, q0 + in_off[i], p0 + in_off[i], h[i], nsteps[i], stride[i],
                           max_iter, flags, q_out + out_off[i], p_out + out_off[i], NULL, NULL,
                           &st);
    if (iters_total) iters_total[i] = st.iterations;
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

/* The same for the s-stage member (flags apply to s = 8 only). */
int orc_integrate_batch_s(int32_t n_inst, int32_t s, const orc_problem *probs, const double *q0,
                        const double *p0, const double *h, const int64_t *nsteps,
                        const int64_t *stride, int32_t max_iter, int32_t flags, double *q_out,
                        double *p_out, int64_t *iters_total, int32_t *status) {
  int64_t *in_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  int64_t *out_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  if (!in_off || !out_off) {
    free(in_off);
    free(out_off);
    return ORC_ENOMEM;
  }
  in_off[0] = out_off[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    int64_t Dq = (int64_t)probs[i].n * probs[i].d;
    if (stride[i] < 1 || nsteps[i] < 0 || nsteps[i] % stride[i]) {
      free(in_off);
      free(out_off);
      return ORC_EINVAL;
    }
    in_off[i + 1] = in_off[i] + Dq;
    out_off[i + 1] = out_off[i] + Dq * (nsteps[i] / stride[i] + 1);
  }
  int worst = ORC_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_inst; ++i) {
    orc_stats st;
    int rc = s == S ? orc_integrate(probs + i, q0 + in_off[i], p0 + in_off[i], h[i], nsteps[i],
                                    stride[i], max_iter, flags, q_out + out_off[i],
                                    p_out + out_off[i], NULL, NULL, &st)
                    : orc_integrate_s(probs + i, s, q0 + in_off[i], p0 + in_off[i], h[i],
                                      nsteps[i], stride[i], max_iter, q_out + out_off[i],
                                      p_out + out_off[i], NULL, &st);
    if (iters_total) iters_total[i] = st.iterations;
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

/* Table access for pins (read-only copies). */
void orc_tableau(double *c, double *b, double *eta, double *mu, double *nu) {
  for (int i = 0; i < S; ++i) {
    c[i] = ORC_C[i];
    b[i] = ORC_B[i];
    for (int j = 0; j < S; ++j) {
      eta[i * S + j] = ORC_ETA[i][j];
      mu[i * S + j] = ORC_MU[i][j];
      nu[i * S + j] = ORC_NU[i][j];
    }
  }
}

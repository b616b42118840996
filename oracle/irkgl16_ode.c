/*
 * Plain FP64 oracle for fixed-step IRKGL16 in the floating-point-symplectic
 * FIRST-ORDER (mu) formulation, for y' = f(t, y) with y in R^D (and, with
 * orc_integrate_ode_s, the s-stage members s = 2, 4, 6: s in place of 8).
 *
 * TEST INFRASTRUCTURE ONLY.  Like irkgl16_oracle.c it shares no code, header,
 * table or helper with the GPU library; only the test-suite, the smoke check
 * and the benchmark's CPU-baseline leg may load it.  Build flags as there
 * (strict IEEE binary64: no contraction into fma, no reassociation).
 *
 * What one step n computes (paper section 2.4, eqs. Yi2 and yn2; section 2.5,
 * eqs. IRK_init and IRK_FP; stopping rule eq. stopping over all D components):
 *   initial guess:   Y_i = y + sum_j nu_ij L_prev_j          (eq. IRK_init)
 *   iteration k = 1, 2, ...:
 *       F_i  = f(t_i, Y_i),  t_i = fl(fl((n-1) h) + fl(c_i h))
 *       L_i  = hb_i F_i                                        (hb_i = fl(h b_i))
 *       Yn_i = y + sum_j mu_ij L_j                              (eq. IRK_FP)
 *       Delta^l = max_i |Yn_i^l - Y_i^l|;  Y = Yn;  stop test per component
 *   update (eq. yn2, compensated): S = sum_i L_i;  y <- y (+) S;  L_prev <- L
 * with y kept as a two-double value (hi, lo) and x (+) d the same two-double
 * addition as in the second-order oracle.  Stage values use y.hi only; L_prev
 * = 0 on the first step; the L that drives the update is the last computed
 * one, so a step costs exactly 8k evaluations of f.  All sums run from zero in
 * ascending index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tableau.h"

#define S 8

/* problem record: same layout as orc_problem in irkgl16_oracle.c */
typedef struct {
  int32_t kind, n, d;
  const double *mass;
  const double *coupling;
  double G, eps, beta;
} ode_problem;

typedef struct {
  int64_t steps_done;
  int64_t iterations;
  int32_t max_k;
  int32_t nonconverged;
  int32_t status;
} ode_stats;

enum {
  ODE_OSC = 20,     /* y = (q, p), D = 2d: q' = p, p' = -G q                    */
  ODE_KEPLER = 21,  /* y = (q, p), D = 2d: q' = p, p' = -G q / |q|^3            */
  ODE_DAMPED = 22,  /* y = (x, u), D = 2:  x' = u, u' = -x - beta u  (not Hamiltonian) */
  ODE_SBH = 23,     /* y = (r, theta, p_r, p_theta): the charged particle near a
                       Schwarzschild black hole in a magnetic field of section
                       5.1.1 (eq. Ham_SBH); E = G, L = eps, beta = beta       */
  ODE_DRIVEN = 24,  /* y = (x, u), D = 2:  x' = u, u' = G cos t                 */
};

enum { ODE_OK = 0, ODE_EINVAL = -1, ODE_ENOMEM = -2, ODE_ENONFINITE = -4 };

void orc_dw_add(double *hi, double *lo, double delta);
int orc_stop_component(double delta, double *mind, double *prev);

/* tables of the s-stage member (defined in irkgl16_oracle.c) */
typedef struct {
  int s;
  const double *c, *b, *eta, *mu, *nu;
} orc_tab;
int orc_stage_tables(int s, orc_tab *T);

static int ode_dim(const ode_problem *p) { return p->n * p->d; }

static int ode_valid(const ode_problem *p) {
  if (p->n < 1 || p->d < 1) return 0;
  switch (p->kind) {
  case ODE_OSC: return p->n == 2;
  case ODE_KEPLER: return p->n == 2;
  case ODE_DAMPED: return ode_dim(p) == 2;
  case ODE_SBH: return ode_dim(p) == 4;
  case ODE_DRIVEN: return ode_dim(p) == 2;
  }
  return 0;
}

/* f(t, Y) */
void orc_rhs(const ode_problem *p, double t, const double *Y, double *F) {
  const int D = ode_dim(p);
  (void)t;
  switch (p->kind) {
  case ODE_OSC: {
    const int d = D / 2;
    for (int k = 0; k < d; ++k) {
      F[k] = Y[d + k];
      F[d + k] = -p->G * Y[k];
    }
    break;
  }
  case ODE_KEPLER: {
    const int d = D / 2;
    double r2 = 0.0;
    for (int k = 0; k < d; ++k) r2 += Y[k] * Y[k];
    double r3 = r2 * sqrt(r2);
    for (int k = 0; k < d; ++k) {
      F[k] = Y[d + k];
      F[d + k] = -p->G * Y[k] / r3;
    }
    break;
  }
  case ODE_DAMPED:
    F[0] = Y[1];
    F[1] = -Y[0] - p->beta * Y[1];
    break;
  case ODE_DRIVEN:
    F[0] = Y[1];
    F[1] = p->G * cos(t);
    break;
  case ODE_SBH: {
    /* H = (1-2/r) p_r^2 / 2 - E^2 / (2 (1-2/r)) + p_th^2 / (2 r^2)
     *     + (L - beta r^2 sin^2 th / 2)^2 / (2 r^2 sin^2 th);
     * y' = (dH/dp_r, dH/dp_th, -dH/dr, -dH/dth), written out with
     * A = 1 - 2/r, s = sin th, c = cos th:
     *   dH/dr  = p_r^2/r^2 + E^2/(r^2 A^2) - p_th^2/r^3 - L^2/(r^3 s^2) + beta^2 r s^2/4
     *   dH/dth = -L^2 c/(r^2 s^3) + beta^2 r^2 s c/4 */
    const double E = p->G, L = p->eps, b = p->beta;
    const double r = Y[0], th = Y[1], pr = Y[2], pth = Y[3];
    const double A = 1.0 - 2.0 / r;
    const double s = sin(th), c = cos(th);
    const double r2 = r * r, r3 = r2 * r, s2 = s * s;
    F[0] = A * pr;
    F[1] = pth / r2;
    F[2] = -(pr * pr / r2 + E * E / (r2 * (A * A)) - pth * pth / r3 - L * L / (r3 * s2) +
             b * b * r * s2 / 4.0);
    F[3] = L * L * c / (r2 * (s2 * s)) - b * b * r2 * s * c / 4.0;
    break;
  }
  }
}

/* H(y) of the Hamiltonian kinds; the damped and driven kinds return (x^2 + u^2)/2. */
double orc_energy_ode(const ode_problem *p, const double *y) {
  const int D = ode_dim(p);
  switch (p->kind) {
  case ODE_OSC: {
    const int d = D / 2;
    double T = 0.0, U = 0.0;
    for (int k = 0; k < d; ++k) {
      T += 0.5 * y[d + k] * y[d + k];
      U += 0.5 * p->G * y[k] * y[k];
    }
    return T + U;
  }
  case ODE_KEPLER: {
    const int d = D / 2;
    double T = 0.0, r2 = 0.0;
    for (int k = 0; k < d; ++k) {
      T += 0.5 * y[d + k] * y[d + k];
      r2 += y[k] * y[k];
    }
    return T - p->G / sqrt(r2);
  }
  case ODE_DAMPED:
  case ODE_DRIVEN:
    return 0.5 * (y[0] * y[0] + y[1] * y[1]);
  case ODE_SBH: {
    const double E = p->G, L = p->eps, b = p->beta;
    const double r = y[0], th = y[1], pr = y[2], pth = y[3];
    const double A = 1.0 - 2.0 / r;
    const double s = sin(th);
    const double u = r * r * s * s;
    const double w = L - 0.5 * b * u;
    return 0.5 * A * pr * pr - 0.5 * E * E / A + pth * pth / (2.0 * r * r) + w * w / (2.0 * u);
  }
  }
  return NAN;
}

/*
 * Integrate one instance.  y0: D values.  Frames f = 0..nsteps/stride (state
 * after f*stride steps; frame 0 is y0) are written to y_out as [frame][D]
 * (y.hi).  iters (nullable): k of each step.  After a non-finite Delta the
 * instance stops and its remaining frames are NaN.
 */
static int ode_core(const ode_problem *p, const orc_tab *T, const double *y0, double h,
                    int64_t nsteps, int64_t stride, int32_t max_iter, double *y_out,
                    int32_t *iters, ode_stats *st) {
  if (!ode_valid(p) || !isfinite(h) || nsteps < 0 || stride < 1 || nsteps % stride ||
      max_iter < 1)
    return ODE_EINVAL;
  const int D = ode_dim(p);
  const int s = T->s;
  const double *mu = T->mu, *nu = T->nu;
  double *buf = (double *)calloc((size_t)D * (4 + 4 * s), sizeof(double));
  if (!buf) return ODE_ENOMEM;
  double *yh = buf, *yl = yh + D, *mind = yl + D, *prev = mind + D;
  double *Y = prev + D, *Yn = Y + s * D, *L = Yn + s * D, *Lp = L + s * D;
  double F[64];
  if (D > 64) {
    free(buf);
    return ODE_EINVAL;
  }
  double hb[S];
  for (int i = 0; i < s; ++i) hb[i] = h * T->b[i];
  for (int l = 0; l < D; ++l) {
    yh[l] = y0[l];
    y_out[l] = y0[l];
  }
  ode_stats loc = {0, 0, 0, 0, ODE_OK};
  int dead = 0;
  for (int64_t n = 1; n <= nsteps; ++n) {
    if (!dead) {
      /* initial guess: Y_i = y + sum_j nu_ij L_prev_j */
      for (int i = 0; i < s; ++i)
        for (int l = 0; l < D; ++l) {
          double sum = 0.0;
          for (int j = 0; j < s; ++j) sum += nu[i * s + j] * Lp[j * D + l];
          Y[i * D + l] = yh[l] + sum;
        }
      for (int l = 0; l < D; ++l) mind[l] = prev[l] = INFINITY;
      int k = 0, conv = 0;
      const double t_prev = (double)(n - 1) * h;
      while (!conv && k < max_iter) {
        ++k;
        for (int i = 0; i < s; ++i) {
          orc_rhs(p, t_prev + T->c[i] * h, Y + i * D, F);
          for (int l = 0; l < D; ++l) L[i * D + l] = hb[i] * F[l];
        }
        for (int i = 0; i < s; ++i)
          for (int l = 0; l < D; ++l) {
            double sum = 0.0;
            for (int j = 0; j < s; ++j) sum += mu[i * s + j] * L[j * D + l];
            Yn[i * D + l] = yh[l] + sum;
          }
        conv = 1;
        for (int l = 0; l < D; ++l) {
          double dl = 0.0;
          for (int i = 0; i < s; ++i) {
            double a = fabs(Yn[i * D + l] - Y[i * D + l]);
            if (isnan(a) || a > dl) dl = a;
          }
          if (!isfinite(dl)) dead = 1;
          if (!orc_stop_component(dl, mind + l, prev + l)) conv = 0;
        }
        memcpy(Y, Yn, sizeof(double) * s * D);
        if (dead) break;
      }
      if (!dead) {
        if (!conv) ++loc.nonconverged;
        loc.iterations += k;
        if (k > loc.max_k) loc.max_k = k;
        if (iters) iters[n - 1] = k;
        for (int l = 0; l < D; ++l) {
          double sum = 0.0;
          for (int i = 0; i < s; ++i) sum += L[i * D + l];
          orc_dw_add(yh + l, yl + l, sum);
        }
        memcpy(Lp, L, sizeof(double) * s * D);
        loc.steps_done = n;
      } else {
        loc.status = ODE_ENONFINITE;
      }
    }
    if (n % stride == 0) {
      double *yo = y_out + (n / stride) * D;
      for (int l = 0; l < D; ++l) yo[l] = dead ? NAN : yh[l];
    }
  }
  if (st) *st = loc;
  free(buf);
  return loc.status;
}

int orc_integrate_ode(const ode_problem *p, const double *y0, double h, int64_t nsteps,
                      int64_t stride, int32_t max_iter, double *y_out, int32_t *iters,
                      ode_stats *st) {
  orc_tab T;
  orc_stage_tables(S, &T);
  return ode_core(p, &T, y0, h, nsteps, stride, max_iter, y_out, iters, st);
}

/* The same with the s-stage member of the family (s = 2, 4, 6, 8). */
int orc_integrate_ode_s(const ode_problem *p, int32_t s, const double *y0, double h,
                        int64_t nsteps, int64_t stride, int32_t max_iter, double *y_out,
                        int32_t *iters, ode_stats *st) {
  orc_tab T;
  if (!orc_stage_tables(s, &T)) return ODE_EINVAL;
  return ode_core(p, &T, y0, h, nsteps, stride, max_iter, y_out, iters, st);
}

/* Many instances (OpenMP over instances); packed as the GPU library packs
 * them: y0 concatenated, frames [frame][D] per instance in order. */
int orc_integrate_ode_batch(int32_t n_inst, const ode_problem *probs, const double *y0,
                            const double *h, const int64_t *nsteps, const int64_t *stride,
                            int32_t max_iter, double *y_out, int64_t *iters_total,
                            int32_t *status) {
  int64_t *in_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  int64_t *out_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  if (!in_off || !out_off) {
    free(in_off);
    free(out_off);
    return ODE_ENOMEM;
  }
  in_off[0] = out_off[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    const int64_t D = (int64_t)probs[i].n * probs[i].d;
    if (stride[i] < 1 || nsteps[i] < 0 || nsteps[i] % stride[i]) {
      free(in_off);
      free(out_off);
      return ODE_EINVAL;
    }
    in_off[i + 1] = in_off[i] + D;
    out_off[i + 1] = out_off[i] + D * (nsteps[i] / stride[i] + 1);
  }
  int worst = ODE_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_inst; ++i) {
    ode_stats st;
    int rc = orc_integrate_ode(probs + i, y0 + in_off[i], h[i], nsteps[i], stride[i], max_iter,
                               y_out + out_off[i], NULL, &st);
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

/* The same for the s-stage member. */
int orc_integrate_ode_batch_s(int32_t n_inst, int32_t s, const ode_problem *probs, const double *y0,
                            const double *h, const int64_t *nsteps, const int64_t *stride,
                            int32_t max_iter, double *y_out, int64_t *iters_total,
                            int32_t *status) {
  int64_t *in_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  int64_t *out_off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_inst + 1));
  if (!in_off || !out_off) {
    free(in_off);
    free(out_off);
    return ODE_ENOMEM;
  }
  in_off[0] = out_off[0] = 0;
  for (int i = 0; i < n_inst; ++i) {
    const int64_t D = (int64_t)probs[i].n * probs[i].d;
    if (stride[i] < 1 || nsteps[i] < 0 || nsteps[i] % stride[i]) {
      free(in_off);
      free(out_off);
      return ODE_EINVAL;
    }
    in_off[i + 1] = in_off[i] + D;
    out_off[i + 1] = out_off[i] + D * (nsteps[i] / stride[i] + 1);
  }
  int worst = ODE_OK;
#pragma omp parallel for schedule(dynamic, 1)
  for (int i = 0; i < n_inst; ++i) {
    ode_stats st;
    int rc = orc_integrate_ode_s(probs + i, s, y0 + in_off[i], h[i], nsteps[i], stride[i],
                                 max_iter, y_out + out_off[i], NULL, &st);
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

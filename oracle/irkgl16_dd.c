/*
 * Double-double oracle for IRKGL16 (second-order eta form): the same steps as
 * the FP64 oracle, carried out in double-double arithmetic (~106-bit
 * significands) with double-double coefficient tables.  It provides
 * reference trajectories whose own rounding error is ~1e-30, far below the
 * FP64 integrator's.
 *
 * TEST INFRASTRUCTURE ONLY; shares no code with the GPU library.
 *
 * Double-double primitives follow the published methods: TwoSum (Knuth),
 * Fast2Sum (Dekker 1971), TwoProd with a fused multiply-add, and the
 * accurate double-double addition, multiplication and long division of
 * Hida, Li and Bailey ("Algorithms for quad-double precision floating point
 * arithmetic", 2001); the square root uses one Karp-Markstein correction of
 * the binary64 square root.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "tableau.h"

#define S 8

typedef struct { double hi, lo; } dd;

static inline dd two_sum(double a, double b) {
  double s = a + b, bb = s - a;
  dd r = {s, (a - (s - bb)) + (b - bb)};
  return r;
}
static inline dd fast_two_sum(double a, double b) {
  double s = a + b;
  dd r = {s, b - (s - a)};
  return r;
}
static inline dd two_prod(double a, double b) {
  double p = a * b;
  dd r = {p, fma(a, b, -p)};
  return r;
}
static inline dd mk(double x) { dd r = {x, 0.0}; return r; }
static inline dd add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi), t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
static inline dd neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }
static inline dd sub(dd a, dd b) { return add(a, neg(b)); }
static inline dd mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
static inline dd muld(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return fast_two_sum(p.hi, p.lo);
}
static inline dd divv(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = sub(a, muld(b, q1));
  double q2 = r.hi / b.hi;
  r = sub(r, muld(b, q2));
  double q3 = r.hi / b.hi;
  dd q = fast_two_sum(q1, q2);
  return add(q, mk(q3));
}
static inline dd ddsqrt(dd a) {
  if (a.hi <= 0.0) return mk(sqrt(a.hi));
  double x = 1.0 / sqrt(a.hi);
  double y = a.hi * x;
  dd y2 = two_prod(y, y);
  double corr = sub(a, y2).hi * (x * 0.5);
  return two_sum(y, corr);
}
static inline dd ddabs(dd a) { return a.hi < 0.0 ? neg(a) : a; }
static inline int lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

enum { K_KEPLER = 0, K_GRAVITY = 1, K_CHAIN = 2, K_HARMONIC = 10, K_CONST = 11, K_HENON = 12 };

typedef struct {
  int32_t kind, n, d;
  const double *mass;
  const double *coupling;
  double G, eps, beta;
} ddo_problem;

static double mass_of(const ddo_problem *p, int body) {
  if (p->kind == K_GRAVITY) return p->mass[body];
  if (p->kind == K_CHAIN) return p->mass ? p->mass[body] : 1.0;
  return 1.0;
}

static dd dV(dd s, double beta) { return add(s, muld(mul(mul(s, s), s), beta)); }

static void force(const ddo_problem *p, const dd *Q, dd *G) {
  const int n = p->n, d = p->d, Dq = n * d;
  switch (p->kind) {
  case K_KEPLER: {
    dd r2 = mk(0.0);
    for (int k = 0; k < Dq; ++k) r2 = add(r2, mul(Q[k], Q[k]));
    dd r3 = mul(r2, ddsqrt(r2));
    for (int k = 0; k < Dq; ++k) G[k] = neg(divv(muld(Q[k], p->G), r3));
    break;
  }
  case K_GRAVITY: {
    dd eps2 = two_prod(p->eps, p->eps);
    for (int a = 0; a < n; ++a) {
      dd acc[3] = {{0, 0}, {0, 0}, {0, 0}};
      for (int b = 0; b < n; ++b) {
        if (b == a) continue;
        dd dx[3], r2 = mk(0.0);
        for (int k = 0; k < d; ++k) {
          dx[k] = sub(Q[b * d + k], Q[a * d + k]);
          r2 = add(r2, mul(dx[k], dx[k]));
        }
        r2 = add(r2, eps2);
        dd w = divv(mk(p->mass[b]), mul(r2, ddsqrt(r2)));
        for (int k = 0; k < d; ++k) acc[k] = add(acc[k], mul(w, dx[k]));
      }
      for (int k = 0; k < d; ++k) G[a * d + k] = muld(acc[k], p->G);
    }
    break;
  }
  case K_CHAIN:
    for (int i = 0; i < n; ++i) {
      dd ql = (i > 0) ? Q[i - 1] : mk(0.0);
      dd qr = (i < n - 1) ? Q[i + 1] : mk(0.0);
      double kl = p->coupling ? p->coupling[i] : 1.0;
      double kr = p->coupling ? p->coupling[i + 1] : 1.0;
      dd F = sub(muld(dV(sub(qr, Q[i]), p->beta), kr), muld(dV(sub(Q[i], ql), p->beta), kl));
      G[i] = divv(F, mk(mass_of(p, i)));
    }
    break;
  case K_HARMONIC:
    for (int k = 0; k < Dq; ++k) G[k] = neg(muld(Q[k], p->G));
    break;
  case K_CONST:
    for (int k = 0; k < Dq; ++k) G[k] = mk(p->G);
    break;
  case K_HENON:
    G[0] = sub(neg(Q[0]), muld(mul(Q[0], Q[1]), 2.0));
    G[1] = sub(neg(Q[1]), sub(mul(Q[0], Q[0]), mul(Q[1], Q[1])));
    break;
  }
}

static dd tab(const double hi[S][S], const double lo[S][S], int i, int j) {
  dd r = {hi[i][j], lo[i][j]};
  return r;
}

/*
 * Integrate one instance in double-double.  Inputs are binary64; the state,
 * stage values and every sum are double-double.  Frames as in the FP64
 * oracle, written as hi and lo parts ([frame][Dq]).  Same stopping rule,
 * evaluated on double-double differences.
 */
int ddo_integrate(const ddo_problem *p, const double *q0, const double *p0, double h,
                  int64_t nsteps, int64_t stride, int32_t max_iter, double *q_hi, double *q_lo,
                  double *p_hi, double *p_lo, int32_t *iters) {
  if (stride < 1 || nsteps < 0 || nsteps % stride || max_iter < 1) return -1;
  const int Dq = p->n * p->d;
  dd *buf = (dd *)calloc((size_t)Dq * (4 + 6 * S), sizeof(dd));
  if (!buf) return -2;
  dd *q = buf, *v = q + Dq, *mind = v + Dq, *prev = mind + Dq;
  dd *Q = prev + Dq, *Qn = Q + S * Dq, *G = Qn + S * Dq, *R = G + S * Dq, *Rp = R + S * Dq,
     *V0 = Rp + S * Dq;
  dd hb[S], hdd = mk(h), c[S];
  for (int i = 0; i < S; ++i) {
    dd bi = {ORC_DD_B_HI[i], ORC_DD_B_LO[i]};
    hb[i] = mul(hdd, bi);
    c[i].hi = ORC_DD_C_HI[i];
    c[i].lo = ORC_DD_C_LO[i];
  }
  for (int l = 0; l < Dq; ++l) {
    q[l] = mk(q0[l]);
    v[l] = divv(mk(p0[l]), mk(mass_of(p, l / p->d)));
  }
  int64_t frame = 0;
  for (int l = 0; l < Dq; ++l) {
    dd pm = muld(v[l], mass_of(p, l / p->d));
    q_hi[l] = q[l].hi; q_lo[l] = q[l].lo; p_hi[l] = pm.hi; p_lo[l] = pm.lo;
  }
  int rc = 0;
  for (int64_t n = 1; n <= nsteps; ++n) {
    for (int i = 0; i < S; ++i)
      for (int l = 0; l < Dq; ++l) {
        dd s = mk(0.0);
        for (int j = 0; j < S; ++j) s = add(s, mul(tab(ORC_DD_NU_HI, ORC_DD_NU_LO, i, j), Rp[j * Dq + l]));
        V0[i * Dq + l] = add(v[l], s);
      }
    for (int i = 0; i < S; ++i)
      for (int l = 0; l < Dq; ++l) {
        dd s = mk(0.0);
        for (int j = 0; j < S; ++j)
          s = add(s, mul(tab(ORC_DD_MU_HI, ORC_DD_MU_LO, i, j), mul(hb[j], V0[j * Dq + l])));
        Q[i * Dq + l] = add(q[l], s);
      }
    for (int l = 0; l < Dq; ++l) mind[l] = prev[l] = mk(INFINITY);
    int k = 0, conv = 0, bad = 0;
    while (!conv && k < max_iter) {
      ++k;
      for (int i = 0; i < S; ++i) force(p, Q + i * Dq, G + i * Dq);
      for (int i = 0; i < S; ++i)
        for (int l = 0; l < Dq; ++l) R[i * Dq + l] = mul(hb[i], G[i * Dq + l]);
      for (int i = 0; i < S; ++i)
        for (int l = 0; l < Dq; ++l) {
          dd s = mk(0.0);
          for (int j = 0; j < S; ++j)
            s = add(s, mul(tab(ORC_DD_ETA_HI, ORC_DD_ETA_LO, i, j), R[j * Dq + l]));
          Qn[i * Dq + l] = add(q[l], mul(hdd, add(mul(c[i], v[l]), s)));
        }
      conv = 1;
      for (int l = 0; l < Dq; ++l) {
        dd dl = mk(0.0);
        for (int i = 0; i < S; ++i) {
          dd a = ddabs(sub(Qn[i * Dq + l], Q[i * Dq + l]));
          if (isnan(a.hi) || lt(dl, a)) dl = a;
        }
        if (!isfinite(dl.hi)) bad = 1;
        if (isnan(dl.hi)) { bad = 1; }
        dd m = lt(prev[l], dl) ? prev[l] : dl;
        int ok = (dl.hi == 0.0 && dl.lo == 0.0) || !lt(m, mind[l]);
        if (lt(prev[l], mind[l])) mind[l] = prev[l];
        prev[l] = dl;
        if (!ok) conv = 0;
      }
      memcpy(Q, Qn, sizeof(dd) * S * Dq);
      if (bad) break;
    }
    if (iters) iters[n - 1] = k;
    if (bad) { rc = -4; break; }
    if (!conv) rc = 1;
    for (int l = 0; l < Dq; ++l) {
      dd sv = mk(0.0), sc = mk(0.0);
      for (int i = 0; i < S; ++i) sv = add(sv, R[i * Dq + l]);
      for (int i = 0; i < S; ++i) sc = add(sc, mul(c[i], R[i * Dq + l]));
      v[l] = add(v[l], sv);
      q[l] = add(q[l], mul(hdd, sub(v[l], sc)));
    }
    memcpy(Rp, R, sizeof(dd) * S * Dq);
    if (n % stride == 0) {
      ++frame;
      for (int l = 0; l < Dq; ++l) {
        dd pm = muld(v[l], mass_of(p, l / p->d));
        q_hi[frame * Dq + l] = q[l].hi; q_lo[frame * Dq + l] = q[l].lo;
        p_hi[frame * Dq + l] = pm.hi; p_lo[frame * Dq + l] = pm.lo;
      }
    }
  }
  free(buf);
  return rc;
}

/* Double-double Hamiltonian of the state (q_hi + q_lo, p_hi + p_lo). */
void ddo_energy(const ddo_problem *pr, const double *qh, const double *ql, const double *ph,
                const double *pl, double *H_hi, double *H_lo) {
  const int n = pr->n, d = pr->d, Dq = n * d;
  dd *q = (dd *)malloc(sizeof(dd) * Dq), *pp = (dd *)malloc(sizeof(dd) * Dq);
  for (int l = 0; l < Dq; ++l) { q[l].hi = qh[l]; q[l].lo = ql[l]; pp[l].hi = ph[l]; pp[l].lo = pl[l]; }
  dd T = mk(0.0), U = mk(0.0);
  for (int a = 0; a < n; ++a)
    for (int k = 0; k < d; ++k)
      T = add(T, divv(mul(pp[a * d + k], pp[a * d + k]), mk(2.0 * mass_of(pr, a))));
  switch (pr->kind) {
  case K_KEPLER: {
    dd r2 = mk(0.0);
    for (int k = 0; k < Dq; ++k) r2 = add(r2, mul(q[k], q[k]));
    U = neg(divv(mk(pr->G), ddsqrt(r2)));
    break;
  }
  case K_GRAVITY: {
    dd eps2 = two_prod(pr->eps, pr->eps);
    for (int a = 0; a < n; ++a)
      for (int b = a + 1; b < n; ++b) {
        dd r2 = mk(0.0);
        for (int k = 0; k < d; ++k) {
          dd dx = sub(q[b * d + k], q[a * d + k]);
          r2 = add(r2, mul(dx, dx));
        }
        dd mm = muld(two_prod(pr->mass[a], pr->mass[b]), pr->G);
        U = sub(U, divv(mm, ddsqrt(add(r2, eps2))));
      }
    break;
  }
  case K_CHAIN:
    for (int i = 0; i <= n; ++i) {
      dd ql_ = (i > 0) ? q[i - 1] : mk(0.0), qr = (i < n) ? q[i] : mk(0.0);
      dd s = sub(qr, ql_), s2 = mul(s, s);
      double k = pr->coupling ? pr->coupling[i] : 1.0;
      U = add(U, muld(add(muld(s2, 0.5), muld(mul(s2, s2), 0.25 * pr->beta)), k));
    }
    break;
  case K_HARMONIC:
    for (int k = 0; k < Dq; ++k) U = add(U, muld(mul(q[k], q[k]), 0.5 * pr->G));
    break;
  case K_CONST:
    for (int k = 0; k < Dq; ++k) U = sub(U, muld(q[k], pr->G));
    break;
  case K_HENON: {
    dd a2 = mul(q[0], q[0]), b2 = mul(q[1], q[1]);
    U = add(muld(add(a2, b2), 0.5), sub(mul(a2, q[1]), divv(mul(b2, q[1]), mk(3.0))));
    break;
  }
  }
  dd H = add(T, U);
  *H_hi = H.hi;
  *H_lo = H.lo;
  free(q);
  free(pp);
}

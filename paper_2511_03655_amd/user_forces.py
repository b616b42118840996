"""Device sources of forces for ``irkgl16_create_user``.

Each defines ``irkgl16_user_force(q, g, prm, t)``: it writes the
acceleration g(q, t) = -grad U(q, t) for unit masses at stage time t.  They are written as plain
expressions (the library compiles them with contraction off), so a
reproducible-mode integration performs exactly the operations of the same
expressions evaluated on the CPU.
"""

# Henon-Heiles (paper section 5.1.2): U = (q1^2 + q2^2)/2 + q1^2 q2 - q2^3/3, Dq = 2.
HENON_HEILES = r"""
__device__ void irkgl16_user_force(const double* q, double* g, const double* prm, double t) {
  (void)prm;
  (void)t;
  g[0] = -q[0] - 2.0 * q[0] * q[1];
  g[1] = -q[1] - (q[0] * q[0] - q[1] * q[1]);
}
"""

# Isotropic harmonic oscillator U = w2 |q|^2 / 2, any Dq; prm[0] = w2 per instance.
HARMONIC = r"""
__device__ void irkgl16_user_force(const double* q, double* g, const double* prm, double t) {
  (void)t;
  const double w2 = prm[0];
  for (int k = 0; k < IRKGL16_DQ; ++k) g[k] = -w2 * q[k];
}
"""

# Section 3.3's non-autonomous Henon-Heiles system, Dq = 2:
# g1 = -q1 - 2 a q1 q2, g2 = -q2 - a (q1^2 - q2^2), a = lambda + xi sin t;
# prm = (lambda, xi) per instance.
HENON_HEILES_T = r"""
__device__ void irkgl16_user_force(const double* q, double* g, const double* prm, double t) {
  const double a = prm[0] + prm[1] * sin(t);
  g[0] = -q[0] - 2.0 * a * q[0] * q[1];
  g[1] = -q[1] - a * (q[0] * q[0] - q[1] * q[1]);
}
"""

# Driven particle g = G cos t in every component, any Dq; prm[0] = G.
DRIVEN = r"""
__device__ void irkgl16_user_force(const double* q, double* g, const double* prm, double t) {
  (void)q;
  const double f = prm[0] * cos(t);
  for (int k = 0; k < IRKGL16_DQ; ++k) g[k] = f;
}
"""

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


# ---------------------------------------------------------------- first-order form
# Right-hand sides irkgl16_user_rhs(y, f, prm, t) for irkgl16_create_ode.

# y = (q, p), D = 2d: q' = p, p' = -w2 q; prm[0] = w2.
OSC_RHS = r"""
__device__ void irkgl16_user_rhs(const double* y, double* f, const double* prm, double t) {
  (void)t;
  const int d = IRKGL16_DQ / 2;
  for (int k = 0; k < d; ++k) {
    f[k] = y[d + k];
    f[d + k] = -prm[0] * y[k];
  }
}
"""

# Kepler in (q, p) form, D = 2d: q' = p, p' = -G q / |q|^3; prm[0] = G.
KEPLER_RHS = r"""
__device__ void irkgl16_user_rhs(const double* y, double* f, const double* prm, double t) {
  (void)t;
  const int d = IRKGL16_DQ / 2;
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) r2 += y[k] * y[k];
  const double r3 = r2 * sqrt(r2);
  for (int k = 0; k < d; ++k) {
    f[k] = y[d + k];
    f[d + k] = -prm[0] * y[k] / r3;
  }
}
"""

# Damped oscillator (not Hamiltonian), D = 2: x' = u, u' = -x - beta u; prm[0] = beta.
DAMPED_RHS = r"""
__device__ void irkgl16_user_rhs(const double* y, double* f, const double* prm, double t) {
  (void)t;
  f[0] = y[1];
  f[1] = -y[0] - prm[0] * y[1];
}
"""

# Driven system, D = 2: x' = u, u' = G cos t; prm[0] = G.
DRIVEN_RHS = r"""
__device__ void irkgl16_user_rhs(const double* y, double* f, const double* prm, double t) {
  f[0] = y[1];
  f[1] = prm[0] * cos(t);
}
"""

# Charged particle near a Schwarzschild black hole in a magnetic field
# (section 5.1.1, eq. Ham_SBH), y = (r, theta, p_r, p_theta), D = 4,
# prm = (E, L, beta):  y' = (dH/dp_r, dH/dp_theta, -dH/dr, -dH/dtheta) with
# A = 1 - 2/r, s = sin theta, c = cos theta,
#   dH/dr     = p_r^2/r^2 + E^2/(r^2 A^2) - p_theta^2/r^3 - L^2/(r^3 s^2) + beta^2 r s^2/4,
#   dH/dtheta = -L^2 c/(r^2 s^3) + beta^2 r^2 s c/4.
SCHWARZSCHILD_RHS = r"""
__device__ void irkgl16_user_rhs(const double* y, double* f, const double* prm, double t) {
  (void)t;
  const double E = prm[0], L = prm[1], b = prm[2];
  const double r = y[0], th = y[1], pr = y[2], pth = y[3];
  const double A = 1.0 - 2.0 / r;
  const double s = sin(th), c = cos(th);
  const double r2 = r * r, r3 = r2 * r, s2 = s * s;
  f[0] = A * pr;
  f[1] = pth / r2;
  f[2] = -(pr * pr / r2 + E * E / (r2 * (A * A)) - pth * pth / r3 - L * L / (r3 * s2) +
           b * b * r * s2 / 4.0);
  f[3] = L * L * c / (r2 * (s2 * s)) - b * b * r2 * s * c / 4.0;
}
"""

"""Oracle coefficient tables for the s-stage Gauss-Legendre collocation methods
(s = 8: IRKGL16; s = 2, 4, 6: the lower-order members of the family).

TEST INFRASTRUCTURE ONLY.  Nothing under ``oracle/`` is part of the product
path; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import or run it.  It shares no code with the GPU library.

Everything is computed in multiprecision (mpmath, 120 significant digits) and
rounded to binary64 exactly once, to nearest-even, through ``fractions``:

* nodes ``c_i = (1 + x_i)/2`` with ``x_i`` the zeros of the Legendre polynomial
  of degree 8, found by Newton's method on the three-term recurrence
  (section 2.2, collocation with shifted Gauss-Legendre nodes);
* ``b`` and ``A = (a_ij)`` from the collocation conditions C(s) and B(s)
  (section 2.2), solved as Vandermonde systems;
* IRKN coefficients ``alpha = A^2`` and ``beta_i = sum_k b_k a_ki``
  (section 2.3, eqs. qnvn/Qi);
* the floating-point-symplectic second-order coefficients ``eta``
  (section 2.4, eqs. Gi/Qi2/qnvn2): ``eta_ij = fl(alpha_ij / b_j)`` for j <= i
  and, for i < j, the completion that makes ``eta_ij + c_j = eta_ji + c_i``
  hold exactly (eq. sympl_cond_2).  The printed completion has a sign slip;
  the reading used here is ``eta_ij = c_i - c_j + eta_ji``, evaluated exactly
  on the binary64 values and asserted to be representable;
* the first-order coefficients ``mu`` (section 2.4, eqs. Yi2/yn2):
  ``mu_ij = fl(a_ij / b_j)`` for j <= i and ``mu_ij = 1 - mu_ji`` for i < j;
* the extrapolation coefficients ``nu`` (section 2.2, eq. Pol0).  The printed
  moment system is garbled; the reading used here: ``W_ij`` solves
  ``sum_j W_ij (c_j - 1)^(k-1) = c_i^k / k`` (k = 1..8), i.e. the previous
  step's collocation polynomial is integrated from t_{n-1} to t_{n-1}+c_i h
  through its derivative values at the previous nodes (shifted by -1), and
  ``nu_ij = fl(W_ij / b_j)`` because nu multiplies L = h b f.

Run ``python oracle/tableau.py`` to regenerate ``oracle/tableau.h`` (binary64
tables for s = 8 plus double-double hi/lo pairs for the double-double oracle,
and binary64 tables for s = 2, 4, 6).
"""
from __future__ import annotations

import os
from fractions import Fraction

import mpmath

S = 8
STAGES = (2, 4, 6, 8)
DPS = 120


def _legendre_and_derivative(n, x):
    """P_n(x) and P_n'(x) by the three-term recurrence."""
    p0, p1 = mpmath.mpf(1), x
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    dp = n * (x * p1 - p0) / (x * x - 1)
    return p1, dp


def legendre_zeros(n=S):
    """Zeros of P_n on (-1, 1), ascending, by Newton from cosine guesses."""
    zs = []
    for i in range(1, n + 1):
        x = mpmath.cos(mpmath.pi * (i - mpmath.mpf(1) / 4) / (n + mpmath.mpf(1) / 2))
        for _ in range(200):
            p, dp = _legendre_and_derivative(n, x)
            dx = p / dp
            x -= dx
            if abs(dx) < mpmath.mpf(10) ** (-(DPS - 5)):
                break
        zs.append(x)
    return sorted(zs)


def exact_tableau(s=S):
    """High-precision (c, b, A, alpha, beta, W) of the s-stage method as mpmath objects."""
    S = s
    with mpmath.workdps(DPS):
        x = legendre_zeros(S)
        c = [(1 + xi) / 2 for xi in x]
        # B(s): sum_j b_j c_j^(k-1) = 1/k
        V = mpmath.matrix(S, S)
        for k in range(S):
            for j in range(S):
                V[k, j] = c[j] ** k
        b = mpmath.lu_solve(V, mpmath.matrix([mpmath.mpf(1) / (k + 1) for k in range(S)]))
        b = [b[j] for j in range(S)]
        # C(s): sum_j a_ij c_j^(k-1) = c_i^k / k
        A = [[None] * S for _ in range(S)]
        for i in range(S):
            rhs = mpmath.matrix([c[i] ** (k + 1) / (k + 1) for k in range(S)])
            ai = mpmath.lu_solve(V, rhs)
            for j in range(S):
                A[i][j] = ai[j]
        # nu moment system on the previous step's nodes c_j - 1
        Vs = mpmath.matrix(S, S)
        for k in range(S):
            for j in range(S):
                Vs[k, j] = (c[j] - 1) ** k
        W = [[None] * S for _ in range(S)]
        for i in range(S):
            rhs = mpmath.matrix([c[i] ** (k + 1) / (k + 1) for k in range(S)])
            wi = mpmath.lu_solve(Vs, rhs)
            for j in range(S):
                W[i][j] = wi[j]
        alpha = [[mpmath.fsum(A[i][k] * A[k][j] for k in range(S)) for j in range(S)]
                 for i in range(S)]
        beta = [mpmath.fsum(b[k] * A[k][i] for k in range(S)) for i in range(S)]
    return dict(c=c, b=b, A=A, alpha=alpha, beta=beta, W=W)


def mpf_to_fraction(x):
    """Exact rational value of an mpmath binary float."""
    sign, man, exp, _ = mpmath.mpf(x)._mpf_
    man, exp = (-1) ** sign * int(man), int(exp)
    return Fraction(man * 2 ** exp) if exp >= 0 else Fraction(man, 2 ** (-exp))


def rne(x):
    """Round an mpmath value to the nearest binary64 (ties to even).

    CPython's int/int true division is correctly rounded, so float(Fraction)
    is the correctly rounded binary64 value of the exact rational.
    """
    return float(mpf_to_fraction(x))


def dd_split(x):
    """(hi, lo) binary64 pair with hi = rne(x), lo = rne(x - hi)."""
    with mpmath.workdps(DPS):
        hi = rne(x)
        lo = rne(mpmath.mpf(x) - mpmath.mpf(hi))
    return hi, lo


def fp64_tables(ex=None):
    """The binary64 coefficient tables the integrator uses.

    Returns dict with lists: c, b (length s) and eta, mu, nu (s x s, row i =
    stage being formed, column j = stage summed over).
    """
    ex = ex or exact_tableau()
    S = len(ex["c"])
    with mpmath.workdps(DPS):
        c = [rne(v) for v in ex["c"]]
        b = [rne(v) for v in ex["b"]]
        eta = [[0.0] * S for _ in range(S)]
        mu = [[0.0] * S for _ in range(S)]
        nu = [[0.0] * S for _ in range(S)]
        for i in range(S):
            for j in range(i + 1):
                eta[i][j] = rne(ex["alpha"][i][j] / ex["b"][j])
                mu[i][j] = rne(ex["A"][i][j] / ex["b"][j])
        for i in range(S):
            for j in range(S):
                nu[i][j] = rne(ex["W"][i][j] / ex["b"][j])
    for i in range(S):
        for j in range(i + 1, S):
            e = Fraction(c[i]) - Fraction(c[j]) + Fraction(eta[j][i])
            if Fraction(float(e)) != e:
                raise ArithmeticError(f"eta[{i}][{j}] completion not representable")
            eta[i][j] = float(e)
            m = 1 - Fraction(mu[j][i])
            if Fraction(float(m)) != m:
                raise ArithmeticError(f"mu[{i}][{j}] completion not representable")
            mu[i][j] = float(m)
    eta_naive = [[0.0] * S for _ in range(S)]
    with mpmath.workdps(DPS):
        for i in range(S):
            for j in range(S):
                eta_naive[i][j] = rne(ex["alpha"][i][j] / ex["b"][j])
    return dict(c=c, b=b, eta=eta, mu=mu, nu=nu, eta_naive=eta_naive)


def dd_tables(ex=None):
    """Double-double (hi, lo) tables for the double-double oracle.

    The symplectic completion is applied in double-double: for i < j,
    eta_ij = c_i - c_j + eta_ji and mu_ij = 1 - mu_ji, each evaluated at
    DPS digits on the double-double values of the other entries and then
    split again, so that the completion identities hold to ~2^-106.
    """
    ex = ex or exact_tableau()
    with mpmath.workdps(DPS):
        def val(p):
            return mpmath.mpf(p[0]) + mpmath.mpf(p[1])
        c = [dd_split(v) for v in ex["c"]]
        b = [dd_split(v) for v in ex["b"]]
        eta = [[None] * S for _ in range(S)]
        mu = [[None] * S for _ in range(S)]
        nu = [[dd_split(ex["W"][i][j] / ex["b"][j]) for j in range(S)] for i in range(S)]
        for i in range(S):
            for j in range(i + 1):
                eta[i][j] = dd_split(ex["alpha"][i][j] / ex["b"][j])
                mu[i][j] = dd_split(ex["A"][i][j] / ex["b"][j])
        for i in range(S):
            for j in range(i + 1, S):
                eta[i][j] = dd_split(val(c[i]) - val(c[j]) + val(eta[j][i]))
                mu[i][j] = dd_split(1 - val(mu[j][i]))
    return dict(c=c, b=b, eta=eta, mu=mu, nu=nu)


def splitting_coefficients():
    """Explicit symmetric compositions of Strang steps (section 4, eqs. Strang,
    comp_method, high_order_splitting), in the ABA form
    phi^A_{a_{s+1} h} o phi^B_{b_s h} o ... o phi^B_{b_1 h} o phi^A_{a_1 h}:
    a_1 = g_1/2, a_j = (g_{j-1} + g_j)/2, a_{s+1} = g_s/2, b_j = g_j, and the
    drift fractions c_j = a_1 + ... + a_j at which the B flows act.

    * Strang: s = 1, g = (1).
    * SUZ90 (Suzuki 1990, order 4, s = 5): g_1 = g_2 = g_4 = g_5 =
      1 / (4 - 4^(1/3)), g_3 = 1 - 4 g_1 (the composition is consistent, sum
      g = 1, and fourth order, sum g^3 = 0).

    Returns {name: dict(gamma, a, b, c)} with binary64 values (each rounded
    once from DPS digits) plus the exact mpmath gammas under "gamma_exact".
    """
    out = {}
    with mpmath.workdps(DPS):
        g1 = 1 / (4 - mpmath.cbrt(4))
        for name, gam in (("STRANG", [mpmath.mpf(1)]),
                          ("SUZ90", [g1, g1, 1 - 4 * g1, g1, g1])):
            s = len(gam)
            a = [gam[0] / 2] + [(gam[j - 1] + gam[j]) / 2 for j in range(1, s)] + [gam[-1] / 2]
            c = [mpmath.fsum(a[:j + 1]) for j in range(s)]
            out[name] = dict(gamma=[rne(x) for x in gam], a=[rne(x) for x in a],
                             b=[rne(x) for x in gam], c=[rne(x) for x in c], gamma_exact=gam)
    return out


def _emit_header(path, fp, dd, others):
    lines = [
        "/* Generated by oracle/tableau.py -- do not edit.",
        " * Oracle coefficient tables (test infrastructure only).",
        " * Row index i = stage being formed, column j = stage summed over. */",
        "#ifndef ORACLE_TABLEAU_H",
        "#define ORACLE_TABLEAU_H",
    ]

    def vec(name, xs):
        lines.append(f"static const double {name}[8] = {{" + ", ".join(x.hex() for x in xs) + "};")

    def mat(name, m):
        lines.append(f"static const double {name}[8][8] = {{")
        for row in m:
            lines.append("  {" + ", ".join(x.hex() for x in row) + "},")
        lines.append("};")

    def vec_s(name, xs):
        lines.append(f"static const double {name}[{len(xs)}] = {{" + ", ".join(x.hex() for x in xs) + "};")

    def mat_s(name, m):
        lines.append(f"static const double {name}[{len(m)}][{len(m)}] = {{")
        for row in m:
            lines.append("  {" + ", ".join(x.hex() for x in row) + "},")
        lines.append("};")

    vec("ORC_C", fp["c"])
    vec("ORC_B", fp["b"])
    mat("ORC_ETA", fp["eta"])
    mat("ORC_MU", fp["mu"])
    mat("ORC_NU", fp["nu"])
    mat("ORC_ETA_NAIVE", fp["eta_naive"])  # negative control only: no completion
    for nm in ("c", "b"):
        vec(f"ORC_DD_{nm.upper()}_HI", [p[0] for p in dd[nm]])
        vec(f"ORC_DD_{nm.upper()}_LO", [p[1] for p in dd[nm]])
    for nm in ("eta", "mu", "nu"):
        mat(f"ORC_DD_{nm.upper()}_HI", [[p[0] for p in row] for row in dd[nm]])
        mat(f"ORC_DD_{nm.upper()}_LO", [[p[1] for p in row] for row in dd[nm]])
    for name, t in splitting_coefficients().items():  # explicit baselines
        vec_s(f"ORC_{name}_A", t["a"])
        vec_s(f"ORC_{name}_B", t["b"])
        vec_s(f"ORC_{name}_C", t["c"])
    for st, t in others.items():  # lower stage counts (same construction)
        vec_s(f"ORC_S{st}_C", t["c"])
        vec_s(f"ORC_S{st}_B", t["b"])
        mat_s(f"ORC_S{st}_ETA", t["eta"])
        mat_s(f"ORC_S{st}_MU", t["mu"])
        mat_s(f"ORC_S{st}_NU", t["nu"])
    lines.append("#endif")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ex = exact_tableau()
    fp = fp64_tables(ex)
    dd = dd_tables(ex)
    others = {s: fp64_tables(exact_tableau(s)) for s in STAGES if s != S}
    here = os.path.dirname(os.path.abspath(__file__))
    _emit_header(os.path.join(here, "tableau.h"), fp, dd, others)
    print("wrote", os.path.join(here, "tableau.h"))


if __name__ == "__main__":
    main()

"""Generate ``irkgl16_coeffs.h``: the binary64 coefficient tables compiled into
the HIP library.

Route (chosen independently of any other table in the repository):

* Gauss-Legendre nodes by the Golub-Welsch method: eigenvalues of the
  symmetric tridiagonal Jacobi matrix of the Legendre weight (off-diagonal
  k / sqrt(4k^2 - 1)), refined by a few Newton steps on P_8 evaluated from its
  explicit coefficients; shifted to c = (1 + x)/2 (section 2.2).
* b_j = int_0^1 l_j and a_ij = int_0^{c_i} l_j with l_j the Lagrange basis on c
  (the collocation conditions of section 2.2), by exact polynomial algebra on
  the multiprecision nodes.
* alpha = A A (section 2.3) and the extrapolation weights
  W_ij = int_0^{c_i} lt_j with lt_j the Lagrange basis on the previous step's
  nodes c_j - 1 (eq. Pol0).
* eta_ij = fl(alpha_ij / b_j), mu_ij = fl(a_ij / b_j) for j <= i, completed for
  i < j by eta_ij = c_i - c_j + eta_ji and mu_ij = 1 - mu_ji so that the
  symplecticity condition of eq. sympl_cond_2 (and its first-order analogue)
  hold exactly in binary64; nu_ij = fl(W_ij / b_j).
* fl() rounds a 60-significant-digit decimal string with CPython's correctly
  rounded decimal-to-binary conversion; the completions are formed in exact
  rational arithmetic and checked to be representable.

Run: ``python paper_2511_03655_amd/csrc/gen_coeffs.py``.
"""
import os
from fractions import Fraction

import mpmath

S = 8
STAGES = (2, 4, 6, 8)  # members of the family the library can run (order 2s)
mpmath.mp.dps = 100


def fl(x):
    return float(mpmath.nstr(x, 60, strip_zeros=False, min_fixed=-mpmath.inf, max_fixed=mpmath.inf))


def poly_mul(p, q):
    r = [mpmath.mpf(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            r[i + j] += a * b
    return r


def poly_eval(p, x):
    acc = mpmath.mpf(0)
    for a in reversed(p):
        acc = acc * x + a
    return acc


def poly_integral(p, lo, hi):
    return mpmath.fsum(a * (hi ** (k + 1) - lo ** (k + 1)) / (k + 1) for k, a in enumerate(p))


def lagrange_basis(nodes, j):
    p = [mpmath.mpf(1)]
    for m, xm in enumerate(nodes):
        if m != j:
            p = poly_mul(p, [-xm / (nodes[j] - xm), 1 / (nodes[j] - xm)])
    return p


def legendre_coeffs(n):
    """Monomial coefficients of P_n (Bonnet recurrence on coefficient lists)."""
    p0, p1 = [mpmath.mpf(1)], [mpmath.mpf(0), mpmath.mpf(1)]
    for k in range(1, n):
        xp1 = [mpmath.mpf(0)] + p1
        nxt = [((2 * k + 1) * (xp1[i] if i < len(xp1) else 0)
                - k * (p0[i] if i < len(p0) else 0)) / (k + 1) for i in range(k + 2)]
        p0, p1 = p1, nxt
    return p1


def nodes(S=S):
    J = mpmath.matrix(S, S)
    for k in range(1, S):
        J[k - 1, k] = J[k, k - 1] = k / mpmath.sqrt(4 * k * k - 1)
    ev = mpmath.eigsy(J, eigvals_only=True)
    xs = sorted(ev[i] for i in range(S))
    P = legendre_coeffs(S)
    dP = [k * a for k, a in enumerate(P)][1:]
    out = []
    for x in xs:
        for _ in range(8):
            x -= poly_eval(P, x) / poly_eval(dP, x)
        out.append((1 + x) / 2)
    return out


def tables(S=S):
    c = nodes(S)
    L = [lagrange_basis(c, j) for j in range(S)]
    b = [poly_integral(L[j], 0, 1) for j in range(S)]
    A = [[poly_integral(L[j], 0, c[i]) for j in range(S)] for i in range(S)]
    alpha = [[mpmath.fsum(A[i][k] * A[k][j] for k in range(S)) for j in range(S)] for i in range(S)]
    shifted = [cj - 1 for cj in c]
    Lt = [lagrange_basis(shifted, j) for j in range(S)]
    W = [[poly_integral(Lt[j], 0, c[i]) for j in range(S)] for i in range(S)]

    cf = [fl(x) for x in c]
    bf = [fl(x) for x in b]
    eta = [[None] * S for _ in range(S)]
    mu = [[None] * S for _ in range(S)]
    for i in range(S):
        for j in range(i + 1):
            eta[i][j] = fl(alpha[i][j] / b[j])
            mu[i][j] = fl(A[i][j] / b[j])
    for i in range(S):
        for j in range(i + 1, S):
            e = Fraction(cf[i]) - Fraction(cf[j]) + Fraction(eta[j][i])
            m = 1 - Fraction(mu[j][i])
            assert Fraction(float(e)) == e and Fraction(float(m)) == m
            eta[i][j], mu[i][j] = float(e), float(m)
    nu = [[fl(W[i][j] / b[j]) for j in range(S)] for i in range(S)]
    # Initial guess folded into one matrix (used by the fused-arithmetic mode):
    # mu_sj (h b_j)(v + sum_i nu_ji R_i) summed over j equals
    # h (c_s v + sum_i K_si R_i) with K = A W diag(1/b), since mu_sj b_j = a_sj
    # and the rows of A sum to c_s.
    K = [[fl(mpmath.fsum(A[s][j] * W[j][i] for j in range(S)) / b[i]) for i in range(S)]
         for s in range(S)]
    return dict(c=cf, b=bf, eta=eta, mu=mu, nu=nu, K=K)


def splitting_tables():
    """Explicit baselines (section 4): symmetric compositions of Strang steps in
    ABA form, flat [a_1..a_{s+1} | b_1..b_s | c_1..c_s] with a_1 = g_1/2,
    a_j = (g_{j-1} + g_j)/2, a_{s+1} = g_s/2, b_j = g_j and the drift
    fractions c_j = a_1 + ... + a_j.  Strang: g = (1).  SUZ90 (Suzuki 1990):
    g_1 = g_2 = g_4 = g_5 = x with x the real root of 4 x^3 + (1 - 4 x)^3 = 0
    (sum g = 1 and sum g^3 = 0), found by Newton's method; g_3 = 1 - 4 x."""
    x = mpmath.mpf("0.4")
    for _ in range(200):
        f = 4 * x ** 3 + (1 - 4 * x) ** 3
        df = 12 * x ** 2 - 12 * (1 - 4 * x) ** 2
        x -= f / df
    assert abs(4 * x ** 3 + (1 - 4 * x) ** 3) < mpmath.mpf(10) ** -90
    out = {}
    for name, g in (("Strang", [mpmath.mpf(1)]), ("Suz90", [x, x, 1 - 4 * x, x, x])):
        s = len(g)
        a = [g[0] / 2] + [(g[j - 1] + g[j]) / 2 for j in range(1, s)] + [g[-1] / 2]
        c = [mpmath.fsum(a[:j + 1]) for j in range(s)]
        out[name] = [fl(v) for v in a] + [fl(v) for v in g] + [fl(v) for v in c]
    return out


def emit(path):
    t = tables()
    out = ["// Generated by gen_coeffs.py -- do not edit.",
           "// IRKGL16 binary64 coefficients: Gauss-Legendre nodes c and weights b",
           "// (section 2.2), second-order symplectic eta (section 2.4), first-order mu",
           "// (section 2.4), extrapolation nu (eq. Pol0) and the folded initial-guess",
           "// matrix K = A W diag(1/b).  Row = stage formed, column = stage summed over.",
           "#pragma once", "", "namespace irk {", ""]

    def vec(name, v):
        out.append(f"constexpr double {name}[8] = {{" + ", ".join(x.hex() for x in v) + "};")

    def mat(name, m):
        out.append(f"constexpr double {name}[8][8] = {{")
        for r in m:
            out.append("    {" + ", ".join(x.hex() for x in r) + "},")
        out.append("};")
    # Flat table of every member, in the device layout of Tab<s> (device_common.h):
    # [c | b | eta | mu | nu | K], rows of s.
    for st in STAGES:
        ts = t if st == S else tables(st)
        flat = list(ts["c"]) + list(ts["b"])
        for key in ("eta", "mu", "nu", "K"):
            for row in ts[key]:
                flat += list(row)
        out.append(f"constexpr double kTabS{st}[{len(flat)}] = {{")
        for i in range(0, len(flat), 4):
            out.append("    " + ", ".join(x.hex() for x in flat[i:i + 4]) + ",")
        out.append("};")
    for name, flat in splitting_tables().items():
        out.append(f"constexpr double kSplit{name}[{len(flat)}] = {{" +
                   ", ".join(x.hex() for x in flat) + "};")
    vec("kC", t["c"])
    vec("kB", t["b"])
    mat("kEta", t["eta"])
    mat("kMu", t["mu"])
    mat("kNu", t["nu"])
    mat("kK", t["K"])
    out += ["", "}  // namespace irk", ""]
    with open(path, "w") as f:
        f.write("\n".join(out))


if __name__ == "__main__":
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "irkgl16_coeffs.h")
    emit(p)
    print("wrote", p)

"""Pins for the oracle's coefficient tables (section 2.2 collocation conditions,
section 2.4 floating-point symplectic reformulation, eq. Pol0 extrapolation).

Each check is a property the paper or the mathematics fixes and that the
generator does not impose by construction, or an independent published value.
"""
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import tableau as T

S = 8
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def ex():
    return T.exact_tableau()


@pytest.fixture(scope="module")
def fp(ex):
    return T.fp64_tables(ex)


def test_nodes_weights_match_published_table(ex):
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "gauss_legendre_8.txt"))
            if l.strip() and not l.startswith("#")]
    xs = [float(r[0]) for r in rows]
    ws = [float(r[1]) for r in rows]
    x_all = sorted([-x for x in xs] + xs)
    w_all = [ws[xs.index(abs(x))] for x in x_all]
    for i in range(S):
        assert abs(float(ex["c"][i]) - (1 + x_all[i]) / 2) < 1e-15
        assert abs(float(ex["b"][i]) - w_all[i] / 2) < 1e-15


def test_superconvergence_B16(ex):
    # Only B(8) is imposed; B(16) holds because the nodes are Gauss points.
    with mpmath.workdps(T.DPS):
        for k in range(1, 2 * S + 1):
            r = mpmath.fsum(ex["b"][j] * ex["c"][j] ** (k - 1) for j in range(S)) - mpmath.mpf(1) / k
            assert abs(r) < mpmath.mpf(10) ** -100, k
        # and fails at 17: order is exactly 16
        r = mpmath.fsum(ex["b"][j] * ex["c"][j] ** 16 for j in range(S)) - mpmath.mpf(1) / 17
        assert abs(r) > 1e-12


def test_collocation_C8_and_D8(ex):
    with mpmath.workdps(T.DPS):
        A, b, c = ex["A"], ex["b"], ex["c"]
        for i in range(S):
            for k in range(1, S + 1):
                r = mpmath.fsum(A[i][j] * c[j] ** (k - 1) for j in range(S)) - c[i] ** k / k
                assert abs(r) < mpmath.mpf(10) ** -100
        # D(8) is not imposed
        for j in range(S):
            for k in range(1, S + 1):
                r = mpmath.fsum(b[i] * c[i] ** (k - 1) * A[i][j] for i in range(S)) \
                    - b[j] * (1 - c[j] ** k) / k
                assert abs(r) < mpmath.mpf(10) ** -100


def test_symplecticity_conditions(ex):
    # eq. sym (first-order) and eq. sym2 (second-order), not imposed.
    with mpmath.workdps(T.DPS):
        A, b, c, al, be = ex["A"], ex["b"], ex["c"], ex["alpha"], ex["beta"]
        tol = mpmath.mpf(10) ** -100
        for i in range(S):
            assert abs(be[i] - b[i] * (1 - c[i])) < tol
            for j in range(S):
                assert abs(b[i] * A[i][j] + b[j] * A[j][i] - b[i] * b[j]) < tol
                assert abs(b[i] * (be[j] - al[i][j]) - b[j] * (be[i] - al[j][i])) < tol


def test_symmetry_of_nodes_and_weights(ex):
    with mpmath.workdps(T.DPS):
        for i in range(S):
            assert abs(ex["c"][S - 1 - i] - (1 - ex["c"][i])) < mpmath.mpf(10) ** -100
            assert abs(ex["b"][S - 1 - i] - ex["b"][i]) < mpmath.mpf(10) ** -100


def test_fp64_symplectic_identities_hold_exactly(fp):
    c = [Fraction(x) for x in fp["c"]]
    for i in range(S):
        assert fp["mu"][i][i] == 0.5  # a_ii = b_i / 2 for Gauss methods
        for j in range(S):
            # eq. sympl_cond_2, in exact rational arithmetic on the binary64 values
            assert Fraction(fp["eta"][i][j]) + c[j] == Fraction(fp["eta"][j][i]) + c[i]
            if i != j:
                assert Fraction(fp["mu"][i][j]) + Fraction(fp["mu"][j][i]) == 1


def _ulp(x):
    return np.spacing(abs(x))


def test_lower_entries_correctly_rounded(ex, fp):
    with mpmath.workdps(T.DPS):
        for i in range(S):
            for j in range(i + 1):
                for name, exact in (("eta", ex["alpha"][i][j] / ex["b"][j]),
                                    ("mu", ex["A"][i][j] / ex["b"][j])):
                    v = fp[name][i][j]
                    err = abs(mpmath.mpf(v) - exact)
                    assert err <= mpmath.mpf(_ulp(v)) / 2, (name, i, j)
            for j in range(S):
                v = fp["nu"][i][j]
                err = abs(mpmath.mpf(v) - ex["W"][i][j] / ex["b"][j])
                assert err <= mpmath.mpf(_ulp(v)) / 2


def test_completed_entries_approximate_alpha_over_b(ex, fp):
    # The completion (read as eta_ij = c_i - c_j + eta_ji) must still approximate
    # the real alpha_ij / b_j; the sign printed in the paper would miss by O(1e-2).
    with mpmath.workdps(T.DPS):
        for i in range(S):
            for j in range(i + 1, S):
                e = fp["eta"][i][j]
                assert abs(mpmath.mpf(e) - ex["alpha"][i][j] / ex["b"][j]) < 8 * _ulp(1.0)
                m = fp["mu"][i][j]
                assert abs(mpmath.mpf(m) - ex["A"][i][j] / ex["b"][j]) < 8 * _ulp(1.0)
                wrong = float(fp["c"][i] - fp["c"][j] - fp["eta"][j][i])
                assert abs(wrong - float(ex["alpha"][i][j] / ex["b"][j])) > 1e-4


def test_nu_extrapolates_polynomials(ex, fp):
    # sum_j nu_ij b_j p(c_j - 1) = int_0^{c_i} p  for deg p <= 7  (eq. Pol0)
    rng = np.random.default_rng(7)
    with mpmath.workdps(T.DPS):
        for _ in range(5):
            coef = [mpmath.mpf(float(x)) for x in rng.standard_normal(S)]
            for i in range(S):
                ci = ex["c"][i]
                exact = mpmath.fsum(coef[k] * ci ** (k + 1) / (k + 1) for k in range(S))
                approx = mpmath.fsum(
                    mpmath.mpf(fp["nu"][i][j]) * ex["b"][j] *
                    mpmath.fsum(coef[k] * (ex["c"][j] - 1) ** k for k in range(S))
                    for j in range(S))
                # nu is rounded to binary64 and |nu b| ~ 6e3: relative 1e-11 budget
                assert abs(approx - exact) < 1e-11 * (1 + abs(exact)) * 1e1


def test_compiled_table_matches_generator(orc, fp):
    t = orc.tableau()
    assert np.array_equal(t["c"], np.array(fp["c"]))
    assert np.array_equal(t["b"], np.array(fp["b"]))
    for k in ("eta", "mu", "nu"):
        assert np.array_equal(t[k], np.array(fp[k])), k


def test_known_spectral_radii(ex):
    A = np.array([[float(x) for x in r] for r in ex["A"]])
    al = np.array([[float(x) for x in r] for r in ex["alpha"]])
    assert abs(max(abs(np.linalg.eigvals(A))) - 0.08842) < 5e-5
    assert abs(max(abs(np.linalg.eigvals(al))) - 0.007818) < 5e-6

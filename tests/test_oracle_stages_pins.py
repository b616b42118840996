"""Pins of the s-stage members of the family (s = 2, 4, 6: IRKGL4, IRKGL8,
IRKGL12; section 2.2 collocation with s Gauss-Legendre nodes, order 2s) in
the oracle: tables and both integration forms (no GPU involved)."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import tableau as T
from tests import refsol

STAGES = (2, 4, 6)


@pytest.fixture(scope="module")
def tabs():
    out = {}
    for s in STAGES:
        ex = T.exact_tableau(s)
        out[s] = (ex, T.fp64_tables(ex))
    return out


@pytest.mark.parametrize("s", STAGES)
def test_nodes_and_weights_match_library_gauss_legendre(tabs, s):
    """numpy's Gauss-Legendre rule (Golub-Welsch, an independent routine)."""
    ex, fp = tabs[s]
    x, w = np.polynomial.legendre.leggauss(s)
    assert np.allclose(fp["c"], (1 + x) / 2, rtol=0, atol=1e-15)  # numpy: a few ulp
    assert np.allclose(fp["b"], w / 2, rtol=0, atol=1e-15)


@pytest.mark.parametrize("s", STAGES)
def test_order_conditions_and_symplecticity(tabs, s):
    """B(2s) holds and B(2s+1) fails (order exactly 2s), C(s) holds, and the
    symplecticity condition b_i a_ij + b_j a_ji = b_i b_j (eq. sym)."""
    ex, _ = tabs[s]
    with mpmath.workdps(T.DPS):
        b, c, A = ex["b"], ex["c"], ex["A"]
        for k in range(1, 2 * s + 1):
            r = mpmath.fsum(b[j] * c[j] ** (k - 1) for j in range(s)) - mpmath.mpf(1) / k
            assert abs(r) < mpmath.mpf(10) ** -100, k
        r = mpmath.fsum(b[j] * c[j] ** (2 * s) for j in range(s)) - mpmath.mpf(1) / (2 * s + 1)
        assert abs(r) > 1e-10
        for i in range(s):
            for k in range(1, s + 1):
                r = mpmath.fsum(A[i][j] * c[j] ** (k - 1) for j in range(s)) - c[i] ** k / k
                assert abs(r) < mpmath.mpf(10) ** -100
            for j in range(s):
                assert abs(b[i] * A[i][j] + b[j] * A[j][i] - b[i] * b[j]) < mpmath.mpf(10) ** -100


@pytest.mark.parametrize("s", STAGES)
def test_binary64_symplectic_identities_exact(tabs, s):
    """eta_ij + c_j = eta_ji + c_i (eq. sympl_cond_2) and mu_ij + mu_ji = 1,
    exactly, on the binary64 values; lower triangles correctly rounded."""
    ex, fp = tabs[s]
    F = Fraction
    for i in range(s):
        for j in range(s):
            assert F(fp["eta"][i][j]) + F(fp["c"][j]) == F(fp["eta"][j][i]) + F(fp["c"][i])
            if i != j:
                assert F(fp["mu"][i][j]) + F(fp["mu"][j][i]) == 1
        for j in range(i + 1):
            with mpmath.workdps(T.DPS):
                assert fp["mu"][i][j] == T.rne(ex["A"][i][j] / ex["b"][j])
                assert fp["eta"][i][j] == T.rne(ex["alpha"][i][j] / ex["b"][j])


@pytest.mark.parametrize("s", STAGES)
def test_linear_oscillator_is_the_pade_map(orc, s):
    """q'' = -w2 q: every step of the s-stage method is the [s/s] Pade
    approximant of exp(hA), in both forms (second-order eta form and
    first-order mu form)."""
    w2, h, n = 1.3, 0.4, 200
    M = np.array(refsol.gauss_pade_map(w2, h, s=s).tolist(), dtype=float)
    r = orc.integrate_s(orc.Spec(orc.HARMONIC, 1, 1, G=w2), s, [0.8], [0.3], h, n, 1)
    y = np.stack([r["q"][:, 0], r["p"][:, 0]], 1)
    assert np.abs(y[1:] - y[:-1] @ M.T).max() < 5e-16  # a few ulp of O(1) values
    ro = orc.integrate_ode(orc.Spec(orc.ODE_OSC, 2, 1, G=w2), [0.8, 0.3], h, n, 1, s=s)
    assert np.abs(ro["y"][1:] - ro["y"][:-1] @ M.T).max() < 5e-16
    # a different s gives a different map (visible at a larger step)
    Ms = np.array(refsol.gauss_pade_map(w2, 2.0, s=s).tolist(), dtype=float)
    M8 = np.array(refsol.gauss_pade_map(w2, 2.0, s=8).tolist(), dtype=float)
    assert np.abs(Ms - M8).max() > 1e-12


@pytest.mark.parametrize("s,N", [(2, (32, 64)), (4, (16, 32)), (6, (8, 12))])
def test_order_2s_on_kepler(orc, s, N):
    """Global error after one period of the a = 1, e = 0.1 Kepler orbit
    shrinks like h^(2s): the observed order log(e0/e1)/log(N1/N0) is 2s +- 0.5
    (for s = 6 a step ratio of 1.5 keeps both errors above rounding)."""
    e = 0.1
    x0, v0 = 1 - e, np.sqrt((1 + e) / (1 - e))
    errs = []
    for n in N:
        h = 2 * np.pi / n
        r = orc.integrate_s(orc.Spec(orc.KEPLER, 1, 2, G=1.0), s, [x0, 0.0], [0.0, v0], h, n, n)
        q, _ = refsol.kepler_perihelion(x0, v0, mpmath.mpf(2) * mpmath.pi)
        errs.append(max(abs(r["q"][-1][c] - float(q[c])) for c in range(2)))
    ratio = errs[0] / errs[1]
    assert errs[1] > 1e-13, errs  # above rounding
    order = np.log(ratio) / np.log(N[1] / N[0])
    assert abs(order - 2 * s) < 0.5, (errs, order)


def test_eight_stage_default_is_unchanged(orc):
    """orc_integrate_s with s = 8 is IRKGL16 (bit for bit)."""
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    a = orc.integrate(sp, [0.4, 0.0], [0.0, 2.0], 2 * np.pi / 128, 500, 50, want_iters=True)
    b = orc.integrate_s(sp, 8, [0.4, 0.0], [0.0, 2.0], 2 * np.pi / 128, 500, 50, want_iters=True)
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["iters"], b["iters"])

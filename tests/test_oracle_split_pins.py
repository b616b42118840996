"""Pins of the explicit splitting baselines in the oracle (section 4: Strang,
eq. Strang; symmetric compositions, eq. comp_method, in ABA form, eq.
high_order_splitting; SUZ90 = Suzuki 1990, order 4, 5 stages)."""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from oracle import tableau as T
from tests import refsol


def test_suzuki_coefficients_closed_form():
    """sum g = 1 (consistency), sum g^3 = 0 (fourth order of a symmetric
    composition of second-order steps), symmetry; the ABA weights sum to 1
    and the binary64 values are the correctly rounded ones."""
    co = T.splitting_coefficients()
    with mpmath.workdps(T.DPS):
        g = co["SUZ90"]["gamma_exact"]
        assert abs(mpmath.fsum(g) - 1) < mpmath.mpf(10) ** -100
        assert abs(mpmath.fsum(x ** 3 for x in g)) < mpmath.mpf(10) ** -100
        assert all(abs(g[j] - g[4 - j]) < mpmath.mpf(10) ** -100 for j in range(5))
        assert abs(g[0] * (4 - mpmath.cbrt(4)) - 1) < mpmath.mpf(10) ** -100
    for name in ("STRANG", "SUZ90"):
        t = co[name]
        assert abs(sum(Fraction(x) for x in t["a"]) - 1) < Fraction(1, 2 ** 50)
        assert abs(sum(Fraction(x) for x in t["b"]) - 1) < Fraction(1, 2 ** 50)
        # drift fractions: c_j = a_1 + ... + a_j; the middle kick of SUZ90 is at 1/2
    assert co["SUZ90"]["c"][2] == 0.5 and co["STRANG"]["c"][0] == 0.5


def test_strang_on_oscillator_is_the_flow_product(orc):
    """q'' = -w2 q: one Strang step is the matrix product of the exact flows
    A(h/2) B(h) A(h/2) of eq. flowAB."""
    w2, h, n = 1.7, 0.3, 300
    A = np.array([[1.0, h / 2], [0.0, 1.0]])
    B = np.array([[1.0, 0.0], [-w2 * h, 1.0]])
    M = A @ B @ A
    r = orc.split_integrate(orc.Spec(orc.HARMONIC, 1, 1, G=w2), orc.STRANG, [0.8], [0.3], h, n, 1)
    y = np.stack([r["q"][:, 0], r["p"][:, 0]], 1)
    assert np.abs(y[1:] - y[:-1] @ M.T).max() < 5e-16


@pytest.mark.parametrize("method,order", [(1, 2), (2, 4)])
def test_orders_on_kepler(orc, method, order):
    """Global error after one period of the e = 0.1 Kepler orbit ~ h^order."""
    e = 0.1
    x0, v0 = 1 - e, np.sqrt((1 + e) / (1 - e))
    q, _ = refsol.kepler_perihelion(x0, v0, mpmath.mpf(2) * mpmath.pi)
    errs = []
    for n in (64, 128):
        r = orc.split_integrate(orc.Spec(orc.KEPLER, 1, 2, G=1.0), method, [x0, 0.0], [0.0, v0],
                                2 * np.pi / n, n, n)
        errs.append(max(abs(r["q"][-1][c] - float(q[c])) for c in range(2)))
    assert abs(np.log2(errs[0] / errs[1]) - order) < 0.2, errs


@pytest.mark.parametrize("method,order", [(1, 2), (2, 4)])
def test_orders_on_driven_particle(orc, method, order):
    """q'' = G cos t: the kicks act at t_{n-1} + c_j h (the drift fraction);
    a kick at the step's start time would cut the order to 1."""
    G, T_end = 1.3, 10.0
    errs = []
    for n in (100, 200):
        h = T_end / n
        r = orc.split_integrate(orc.Spec(orc.DRIVEN, 1, 1, G=G), method, [0.5], [0.25], h, n, n)
        errs.append(abs(r["q"][-1][0] - (0.5 + 0.25 * T_end + G * (1 - np.cos(T_end)))))
    assert abs(np.log2(errs[0] / errs[1]) - order) < 0.3, errs


def test_suz90_is_the_composition_of_strang_steps(orc):
    """One SUZ90 step equals five Strang steps of sizes g_j h applied in turn
    (eq. comp_method; the ABA form merges adjacent half drifts, so the two
    agree to rounding)."""
    g = T.splitting_coefficients()["SUZ90"]["gamma"]
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    h = 0.2
    q, p = np.array([0.7, 0.1]), np.array([-0.2, 1.2])
    r = orc.split_integrate(sp, orc.SUZ90, q, p, h, 1, 1)
    qq, pp = q, p
    for gj in g:
        rj = orc.split_integrate(sp, orc.STRANG, qq, pp, gj * h, 1, 1)
        qq, pp = rj["q"][-1], rj["p"][-1]
    assert np.abs(r["q"][-1] - qq).max() < 1e-14 and np.abs(r["p"][-1] - pp).max() < 1e-14
    assert np.abs(r["q"][-1] - q).max() > 1e-3  # it moved


@pytest.mark.parametrize("method", [1, 2])
def test_time_reversal_and_bounded_energy(orc, method):
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    e = 0.3
    x0, v0 = 1 - e, np.sqrt((1 + e) / (1 - e))
    h, n = 2 * np.pi / 256, 256 * 40
    r = orc.split_integrate(sp, method, [x0, 0.0], [0.0, v0], h, n, 1)
    back = orc.split_integrate(sp, method, r["q"][-1], r["p"][-1], -h, n, n)
    assert np.abs(back["q"][-1] - [x0, 0.0]).max() < 1e-10
    H = np.array([orc.energy(sp, q, p) for q, p in zip(r["q"], r["p"])])
    dH = np.abs(H - H[0])
    # symplectic: the energy error oscillates within a bound set in the first
    # orbits (the numerical period differs from 2 pi, so samples at fixed
    # times move along that oscillation; only its envelope matters)
    assert dH[n // 2:].max() < 1.05 * dH[:n // 2].max() + 1e-15


def test_update_is_compensated(orc):
    """Free particle, q = 1, v h = 1e-17 per step (below half an ulp of q):
    the two-double state accumulates the drifts."""
    n = 10000
    r = orc.split_integrate(orc.Spec(orc.CONST, 1, 1, G=0.0), orc.SUZ90, [1.0], [1e-17], 1.0, n,
                            n)
    assert r["q"][-1][0] == 1.0 + n * 1e-17 and r["q"][-1][0] > 1.0


def test_velocity_update_is_compensated(orc):
    """Constant acceleration G = 1e-17 on v = 1 with h = 1: each step's kicks
    (sum b_j h G = 1e-17) fall below half an ulp of v; only the two-double
    velocity accumulates them (the last mutation-free digits: within 4 ulp of
    1 + n G)."""
    n, G = 10000, 1e-17
    r = orc.split_integrate(orc.Spec(orc.CONST, 1, 1, G=G), orc.SUZ90, [0.0], [1.0], 1.0, n, n)
    v = r["p"][-1][0]
    assert v > 1.0 and abs(v - (1.0 + n * G)) <= 4 * np.spacing(1.0)

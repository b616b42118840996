"""Pins of the first-order (mu form) FP64 oracle, y' = f(t, y) (section 2.4,
eqs. Yi2 / yn2; section 2.5, eqs. IRK_init / IRK_FP), against what the method
and the mathematics fix (no GPU involved).

A slip in the first-order oracle -- mu and nu exchanged, a missing h b_i, the
wrong update sum, an uncompensated update, a wrong sign or term in a
right-hand side -- fails at least one of these."""
import mpmath
import numpy as np
import pytest

from tests import refsol

KEP_H = 2 * np.pi / 128


def pade_matrix(A, h, s=8, dps=50):
    """One Gauss collocation step on y' = A y: the [s/s] Pade approximant of
    exp(hA) (a textbook property of s-stage Gauss methods), as float."""
    from math import factorial
    with mpmath.workdps(dps):
        p = [mpmath.mpf(factorial(2 * s - k) * factorial(s)) /
             (factorial(2 * s) * factorial(k) * factorial(s - k)) for k in range(s + 1)]
        M = mpmath.matrix(np.asarray(A, float).tolist()) * mpmath.mpf(h)
        n = M.rows

        def P(X):
            acc = mpmath.zeros(n)
            pw = mpmath.eye(n)
            for k in range(s + 1):
                acc += p[k] * pw
                pw = pw * X
            return acc
        R = P(M) * P(-M) ** -1
        return np.array(R.tolist(), dtype=float)


@pytest.mark.parametrize("h", [0.25, 0.5])
def test_ode_oscillator_is_the_pade_map(orc, h):
    """q' = p, p' = -w2 q in first-order form: every step is the [8/8] Pade
    map of exp(hA) to rounding (local error <= 4 ulp-level per step)."""
    w2 = 1.7
    sp = orc.Spec(orc.ODE_OSC, 2, 1, G=w2)
    n = 400
    r = orc.integrate_ode(sp, [1.0, 0.3], h, n, 1, want_iters=True)
    assert r["rc"] == 0
    M = pade_matrix([[0, 1], [-w2, 0]], h)
    y = r["y"]
    loc = np.abs(y[1:] - y[:-1] @ M.T).max()
    assert loc < 1e-15
    # and the whole trajectory against the exact n-step map (mpmath)
    q, v = refsol.pade_trajectory(w2, h, 1.0, 0.3, n)
    assert abs(y[-1, 0] - float(q)) < 1e-13 and abs(y[-1, 1] - float(v)) < 1e-13


def test_ode_damped_system_is_the_pade_map(orc):
    """A non-Hamiltonian linear system y' = A y (damped oscillator), D = 2:
    the method is still the Pade map of exp(hA); with y_n decaying, the
    compensated update keeps every step at rounding level."""
    beta = 0.3
    sp = orc.Spec(orc.ODE_DAMPED, 1, 2, beta=beta)
    A = [[0.0, 1.0], [-1.0, -beta]]
    h, n = 0.4, 300
    r = orc.integrate_ode(sp, [0.7, -0.2], h, n, 1)
    M = pade_matrix(A, h)
    y = r["y"]
    assert np.abs(y[1:] - y[:-1] @ M.T).max() < 1e-16 + 4e-16 * np.abs(y[:-1]).max()
    # Pade vs exp: the method's own error over the run is tiny at this h
    import scipy.linalg
    exact = scipy.linalg.expm(np.array(A) * h * n) @ np.array([0.7, -0.2])
    assert np.abs(y[-1] - exact).max() < 1e-14


def test_ode_kepler_matches_keplers_equation(orc):
    """First-order Kepler (y = (q, p), D = 4) from the perihelion, against the
    closed form, 10^4 steps of 2 pi / 128."""
    sp = orc.Spec(orc.ODE_KEPLER, 2, 2, G=1.0)
    r = orc.integrate_ode(sp, [0.4, 0.0, 0.0, 2.0], KEP_H, 10000, 1000, want_iters=True)
    assert r["rc"] == 0 and r["stats"]["nonconverged"] == 0
    for f in range(r["y"].shape[0]):
        q, v = refsol.kepler_perihelion(0.4, 2.0, mpmath.mpf(KEP_H) * 1000 * f)
        err = max(abs(r["y"][f][c] - float(q[c])) for c in range(2))
        errv = max(abs(r["y"][f][2 + c] - float(v[c])) for c in range(2))
        assert err < 5e-12 and errv < 5e-12, (f, err, errv)


def test_ode_and_second_order_forms_agree(orc):
    """The mu form and the eta form are the same collocation method with
    differently rounded coefficients: after 10^3 Kepler steps they agree at
    rounding level."""
    n = 1000
    a = orc.integrate_ode(orc.Spec(orc.ODE_KEPLER, 2, 2, G=1.0), [0.5, 0.1, -0.3, 1.5], KEP_H,
                          n, n)
    b = orc.integrate(orc.Spec(orc.KEPLER, 1, 2, G=1.0), [0.5, 0.1], [-0.3, 1.5], KEP_H, n, n)
    assert np.abs(a["y"][-1, :2] - b["q"][-1]).max() < 1e-12
    assert np.abs(a["y"][-1, 2:] - b["p"][-1]).max() < 1e-12


def test_ode_stopping_rule_is_applied_literally(orc):
    """Eq. stopping on every component, applied as written: from (q, p) =
    (1, 0) the first iteration leaves q unchanged (its increment uses p = 0),
    the second leaves p unchanged, and so on, so each component has an exact
    zero Delta in its history and the rule stops the first step after 4
    iterations.  From then on the steps are ordinary (rounding-level local
    error against the Pade map)."""
    h = 0.5
    sp = orc.Spec(orc.ODE_OSC, 2, 1, G=1.0)
    r = orc.integrate_ode(sp, [1.0, 0.0], h, 12, 1, want_iters=True)
    assert r["iters"][0] == 4
    M = pade_matrix([[0, 1], [-1, 0]], h)
    y = r["y"]
    assert np.abs(y[1] - M @ y[0]).max() > 1e-6            # truncated first step
    assert np.abs(y[4:] - y[3:-1] @ M.T).max() < 1e-15      # ordinary steps later


def _sbh_initial(orc, E=0.995, L=4.6, beta=8.9e-4, r0=11.0):
    """Section 5.1.1: theta = pi/2, p_r = 0, r = 11, p_theta > 0 from H = -1/2."""
    with mpmath.workdps(40):
        r = mpmath.mpf(r0)
        A = 1 - 2 / r
        w = mpmath.mpf(L) - mpmath.mpf(beta) * r * r / 2
        pth2 = 2 * r * r * (-mpmath.mpf(1) / 2 + mpmath.mpf(E) ** 2 / (2 * A) - w * w / (2 * r * r))
        pth = float(mpmath.sqrt(pth2))
    return orc.Spec(orc.ODE_SBH, 1, 4, G=E, eps=L, beta=beta), np.array([r0, np.pi / 2, 0.0, pth])


def test_ode_schwarzschild_rhs_is_hamiltonian(orc):
    """f = J^{-1} grad H for eq. Ham_SBH, by central differences of H."""
    sp, y0 = _sbh_initial(orc)
    rng = np.random.default_rng(5)
    for _ in range(5):
        y = y0 + rng.normal(0, [1.0, 0.2, 0.05, 0.2])
        f = orc.rhs(sp, 0.0, y)
        g = np.zeros(4)
        for l in range(4):
            e = 1e-6 * max(1.0, abs(y[l]))
            yp, ym = y.copy(), y.copy()
            yp[l] += e
            ym[l] -= e
            g[l] = (orc.energy_ode(sp, yp) - orc.energy_ode(sp, ym)) / (2 * e)
        # (r', th', pr', pth') = (dH/dpr, dH/dpth, -dH/dr, -dH/dth)
        expect = np.array([g[2], g[3], -g[0], -g[1]])
        assert np.allclose(f, expect, rtol=1e-7, atol=1e-9), (f, expect)


def test_ode_schwarzschild_regular_orbit(orc):
    """The paper's regular orbit: H = -1/2 at the start (p_theta from the
    energy condition), energy error at rounding level over 2e4 time units,
    the orbit stays bounded away from the horizon, and integrating back
    returns to the start."""
    sp, y0 = _sbh_initial(orc)
    assert abs(orc.energy_ode(sp, y0) + 0.5) < 1e-15
    h, n = 2.0, 10000
    r = orc.integrate_ode(sp, y0, h, n, 100, want_iters=True)
    assert r["rc"] == 0 and r["stats"]["nonconverged"] == 0
    H = np.array([orc.energy_ode(sp, y) for y in r["y"]])
    assert np.abs(H + 0.5).max() < 2e-14
    assert r["y"][:, 0].min() > 4.0 and r["y"][:, 0].max() < 200.0
    back = orc.integrate_ode(sp, r["y"][-1], -h, n, n)
    assert np.abs(back["y"][-1] - y0).max() < 1e-9


@pytest.mark.parametrize("h", [0.5, -0.25])
def test_ode_driven_follows_closed_form(orc, h):
    """x' = u, u' = G cos t from t = 0: x = x0 + u0 t + G (1 - cos t),
    u = u0 + G sin t.  The stages are evaluated at t_{n-1} + c_i h; any other
    stage time is off by O(h)."""
    G, n = 1.3, 400
    sp = orc.Spec(orc.ODE_DRIVEN, 1, 2, G=G)
    r = orc.integrate_ode(sp, [0.5, 0.25], h, n, 10, want_iters=True)
    t = np.arange(n // 10 + 1) * 10 * h
    assert np.abs(r["y"][:, 0] - (0.5 + 0.25 * t + G * (1 - np.cos(t)))).max() < 1e-12
    assert np.abs(r["y"][:, 1] - (0.25 + G * np.sin(t))).max() < 1e-13


def test_ode_update_is_compensated(orc):
    """q' = p, p' = 0 with q = 1 and p h = 1e-17, below half an ulp of q: a
    plain update would leave q at 1 forever; the two-double state accumulates
    the increments, so after 10^4 steps q.hi = fl(1 + 10^4 * 1e-17)."""
    sp = orc.Spec(orc.ODE_OSC, 2, 1, G=0.0)
    n = 10000
    r = orc.integrate_ode(sp, [1.0, 1e-17], 1.0, n, n)
    assert r["y"][-1, 0] == 1.0 + n * 1e-17
    assert r["y"][-1, 0] > 1.0

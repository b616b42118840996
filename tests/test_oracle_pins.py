"""Pins of the FP64 and double-double oracles against what the method and the
mathematics fix (no GPU involved).

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed coefficient table, a broken compensation or
stopping rule) fails at least one of them.
"""
from fractions import Fraction

import mpmath
import numpy as np
import pytest

from tests import refsol

KEP_H = 2 * np.pi / 128
mpmath.mp.dps = 50  # double-double values are summed at full precision


# ---------------------------------------------------------------- linear problems

@pytest.mark.parametrize("h", [0.25, 0.7])
def test_harmonic_matches_pade_closed_form(orc, h):
    """q'' = -q: each Gauss step is the [8/8] Pade rotation (section 2.2 order 2s)."""
    n = 400
    sp = orc.Spec(orc.HARMONIC, 1, 1, G=1.0)
    r = orc.integrate(sp, [1.0], [0.0], h, n, stride=n)
    qe, ve = refsol.pade_trajectory(1.0, h, 1.0, 0.0, n)
    # roundoff-level agreement: n = 400 steps, phase error ~ sqrt(n) eps
    assert abs(r["q"][-1][0] - float(qe)) < 1e-13
    assert abs(r["p"][-1][0] - float(ve)) < 1e-13
    dd = orc.integrate_dd(sp, [1.0], [0.0], h, n, stride=n)
    assert abs(mpmath.mpf(dd["q_hi"][-1][0]) + dd["q_lo"][-1][0] - qe) < 1e-28
    assert abs(mpmath.mpf(dd["p_hi"][-1][0]) + dd["p_lo"][-1][0] - ve) < 1e-28


def test_linear_chain_modes_are_pade_rotations(orc):
    """A beta = 0 chain is a set of independent normal modes, each rotated by the
    Pade map at its own frequency w_k = 2 sin(k pi / (2(n+1)))."""
    n, h, nsteps = 6, 0.3, 200
    sp = orc.Spec(orc.CHAIN, n, 1, beta=0.0)
    k = 2
    x = np.arange(1, n + 1)
    mode = np.sin(k * np.pi * x / (n + 1))
    r = orc.integrate(sp, 0.01 * mode, np.zeros(n), h, nsteps, stride=nsteps)
    w2 = (2 * np.sin(k * np.pi / (2 * (n + 1)))) ** 2
    qe, ve = refsol.pade_trajectory(w2, h, 0.01, 0.0, nsteps)
    np.testing.assert_allclose(r["q"][-1], float(qe) * mode, atol=1e-15)
    np.testing.assert_allclose(r["p"][-1], float(ve) * mode, atol=1e-15)


# ---------------------------------------------------------------- Kepler (c1)

def _kepler(orc, nsteps, stride):
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    return sp, orc.integrate(sp, [0.4, 0.0], [0.0, 2.0], KEP_H, nsteps, stride=stride,
                             want_iters=True)


def test_kepler_matches_keplers_equation(orc):
    sp, r = _kepler(orc, 10000, 1000)
    for f in range(r["q"].shape[0]):
        q, v = refsol.kepler_perihelion(0.4, 2.0, mpmath.mpf(KEP_H) * 1000 * f)
        err = max(abs(r["q"][f][c] - float(q[c])) for c in range(2))
        assert err < 5e-12, (f, err)
        errv = max(abs(r["p"][f][c] - float(v[c])) for c in range(2))
        assert errv < 5e-12
    assert r["rc"] == 0 and r["stats"]["nonconverged"] == 0


def test_kepler_invariants_to_roundoff(orc):
    sp, r = _kepler(orc, 10000, 10)
    H = np.array([orc.energy(sp, q, p) for q, p in zip(r["q"], r["p"])])
    L = r["q"][:, 0] * r["p"][:, 1] - r["q"][:, 1] * r["p"][:, 0]
    assert np.max(np.abs(H + 0.5)) / 0.5 < 2e-14       # Delta H glob max (eq. DHglobmax)
    assert np.max(np.abs(L - 0.8)) < 2e-14             # quadratic invariant of Gauss methods
    assert 1 <= r["iters"].min() and r["iters"].max() <= 12


@pytest.mark.parametrize("x0", [0.9])
def test_order_sixteen_slope(orc, x0):
    """Global error ~ h^16 (section 2.2): measured with the double-double oracle
    so that rounding does not hide the truncation error."""
    v0 = float(mpmath.sqrt(mpmath.mpf(2) / x0 - 1))  # a = 1
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    T, ks, errs = 5.0, [16, 20, 24, 28, 32], []
    for k in ks:
        h = T / k
        dd = orc.integrate_dd(sp, [x0, 0.0], [0.0, v0], h, k, stride=k)
        q, _ = refsol.kepler_perihelion(x0, v0, mpmath.mpf(h) * k)
        errs.append(float(max(abs(mpmath.mpf(dd["q_hi"][-1][c]) + dd["q_lo"][-1][c] - q[c])
                              for c in range(2))))
    slopes = [np.log(errs[i] / errs[i + 1]) / np.log(ks[i + 1] / ks[i]) for i in range(len(ks) - 1)]
    assert all(15.5 < s < 16.5 for s in slopes), slopes


# ---------------------------------------------------------------- exact cases

def test_free_fall_is_exact_and_converges_in_two(orc):
    """Constant g: collocation is exact, the fixed point is reached after one
    iteration (Delta[2] == 0), and the extrapolated guess is exact from step 2."""
    sp = orc.Spec(orc.CONST, 1, 3, G=-9.81)
    q0, v0, h, n = np.array([0.0, 0.0, 10.0]), np.array([1.0, 0.5, 0.0]), 0.1, 100
    r = orc.integrate(sp, q0, v0, h, n, stride=1, want_iters=True, want_delta1=True)
    assert r["iters"][0] == 2
    assert set(np.unique(r["iters"])) <= {1, 2}
    assert np.all(r["delta1"][1:] < 1e-13)
    assert r["delta1"][0] > 1e-3
    t = np.arange(n + 1)[:, None] * h
    np.testing.assert_allclose(r["q"], q0 + v0 * t - 9.81 * t * t / 2, rtol=0, atol=2e-12)
    np.testing.assert_allclose(r["p"], v0 - 9.81 * t, rtol=0, atol=2e-13)


def test_free_particle_needs_no_force(orc):
    sp = orc.Spec(orc.CONST, 1, 2, G=0.0)
    r = orc.integrate(sp, [1.0, -2.0], [0.25, 0.5], 0.5, 64, stride=64, want_iters=True)
    np.testing.assert_array_equal(r["q"][-1], [1.0 + 0.25 * 32, -2.0 + 0.5 * 32])
    assert r["iters"].max() <= 2


def test_extrapolation_error_scales_with_step(orc):
    """Delta[1] measures the extrapolated guess (eq. IRK_init2): it shrinks much
    faster than h, and switching extrapolation off makes it O(h^2) large."""
    sp = orc.Spec(orc.HARMONIC, 1, 1, G=1.0)
    d = []
    for h in (0.2, 0.1):
        r = orc.integrate(sp, [1.0], [0.0], h, 20, want_delta1=True)
        d.append(np.median(r["delta1"][2:]))
    assert d[0] / d[1] > 2 ** 8   # O(h^9) or better
    r0 = orc.integrate(sp, [1.0], [0.0], 0.1, 20, want_delta1=True,
                       flags=orc.FLAG_NO_EXTRAPOLATION)
    assert np.median(r0["delta1"][2:]) > 1e3 * d[1]


def test_time_reversibility(orc):
    """Symmetric method: n steps with h then n with -h return to the start."""
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    n = 1000
    f = orc.integrate(sp, [0.4, 0.0], [0.0, 2.0], KEP_H, n, stride=n)
    b = orc.integrate(sp, f["q"][-1], f["p"][-1], -KEP_H, n, stride=n)
    tol = 10 * np.sqrt(n) * 2.2e-16 * 2.0 * 10
    assert np.max(np.abs(b["q"][-1] - [0.4, 0.0])) < tol
    assert np.max(np.abs(b["p"][-1] - [0.0, 2.0])) < tol
    # momentum-flip form: reversing p instead of h
    g = orc.integrate(sp, f["q"][-1], -f["p"][-1], KEP_H, n, stride=n)
    assert np.max(np.abs(g["q"][-1] - [0.4, 0.0])) < tol
    assert np.max(np.abs(g["p"][-1] + np.array([0.0, 2.0]))) < tol


# ---------------------------------------------------------------- long-time behaviour

def _ensemble_energy(orc, flags, P=48, n=100000, stride=5000):
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    rng = np.random.default_rng(11)
    q0 = np.tile([0.4, 0.0], (P, 1)) * (1 + 1e-13 * rng.standard_normal((P, 2)))
    p0 = np.tile([0.0, 2.0], (P, 1))
    r = orc.integrate_batch([sp] * P, q0.ravel(), p0.ravel(), KEP_H, n, stride, flags=flags)
    nf = n // stride + 1
    Q, Pm = r["q"].reshape(P, nf, 2), r["p"].reshape(P, nf, 2)
    H = np.array([[orc.energy(sp, Q[i, f], Pm[i, f]) for f in range(nf)] for i in range(P)])
    return (H - H[:, :1]) / np.abs(H[:, :1]), np.arange(nf) * stride


def test_no_energy_drift_and_compensation_matters(orc):
    dH, t = _ensemble_energy(orc, 0)
    m, s = dH.mean(0), dH.std(0)
    P = dH.shape[0]
    assert np.all(np.abs(m[1:]) <= 4 * s[1:] / np.sqrt(P))         # no linear drift
    slope = np.polyfit(np.log(t[1:]), np.log(s[1:]), 1)[0]
    assert 0.3 < slope < 0.8, slope                                  # Brouwer-like sqrt(t)
    assert np.max(np.abs(dH)) < 1e-13
    # negative control: without the two-double state the spread grows markedly
    dHn, _ = _ensemble_energy(orc, orc.FLAG_NO_COMPENSATION)
    assert dHn.std(0)[-1] > 2.5 * s[-1]


def test_henon_heiles_regular_orbit_bounded(orc):
    """Section 5.1.2: q1 = 0, q2 = 0.3, p2 = 0.2, p1 > 0 from H = 1/12."""
    q1, q2, p2 = 0.0, 0.3, 0.2
    p1 = float(mpmath.sqrt(mpmath.mpf(2) / 12 - p2 ** 2 - q1 ** 2 - q2 ** 2
                           - 2 * q1 ** 2 * q2 + mpmath.mpf(2) / 3 * q2 ** 3))
    assert abs(p1 - 0.23380903889000242556) < 1e-16
    sp = orc.Spec(orc.HENON, 1, 2)
    n = 20000
    h = 2 * np.pi / 64
    r = orc.integrate(sp, [q1, q2], [p1, p2], h, n, stride=100)
    H = np.array([orc.energy(sp, q, p) for q, p in zip(r["q"], r["p"])])
    H0 = orc.energy(sp, [q1, q2], [p1, p2])
    assert abs(H0 - 1 / 12) < 1e-16
    assert np.max(np.abs(H - H0)) / H0 < 5e-14
    assert np.max(np.abs(r["q"])) < 1.0


# ---------------------------------------------------------------- FP64 against DD

@pytest.mark.parametrize("case", ["kepler", "nbody", "chain"])
def test_fp64_tracks_double_double(orc, case):
    from paper_2511_03655_amd import workloads as W
    if case == "kepler":
        sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
        q0, p0, h, n, tol = [0.4, 0.0], [0.0, 2.0], KEP_H, 1000, 1e-12
    elif case == "nbody":
        inst = W.planetary_systems(1, n_bodies=6, seed=3)[0]
        sp = orc.Spec(orc.GRAVITY, 6, 3, mass=inst["mass"], G=1.0)
        q0, p0, h, n, tol = inst["q"], inst["p"], 1.0, 1000, 1e-12
    else:
        inst = W.fpu_chain(16, seed=5)
        sp = orc.Spec(orc.CHAIN, 16, 1, beta=1.0)
        q0, p0, h, n, tol = inst["q"], inst["p"], inst["h"], 1000, 1e-12
    f = orc.integrate(sp, q0, p0, h, n, stride=n)
    d = orc.integrate_dd(sp, q0, p0, h, n, stride=n)
    scale = max(np.max(np.abs(d["q_hi"][-1])), 1e-300)
    assert np.max(np.abs(f["q"][-1] - d["q_hi"][-1])) / scale < tol
    pscale = max(np.max(np.abs(d["p_hi"][-1])), 1e-300)
    assert np.max(np.abs(f["p"][-1] - d["p_hi"][-1])) / pscale < tol


# ---------------------------------------------------------------- forces

def test_gravity_force_brute_force_and_momentum(orc):
    rng = np.random.default_rng(2)
    n, d = 7, 3
    m = rng.uniform(0.1, 2.0, n)
    Q = rng.standard_normal(n * d)
    for eps in (0.0, 0.05):
        sp = orc.Spec(orc.GRAVITY, n, d, mass=m, G=0.7, eps=eps)
        G = orc.force(sp, Q)
        with mpmath.workdps(40):
            for a in range(n):
                for k in range(d):
                    acc = mpmath.mpf(0)
                    for b in range(n):
                        if b == a:
                            continue
                        dx = [mpmath.mpf(Q[b * d + j]) - Q[a * d + j] for j in range(d)]
                        r2 = sum(x * x for x in dx) + mpmath.mpf(eps) ** 2
                        acc += mpmath.mpf(m[b]) * dx[k] / r2 ** mpmath.mpf(1.5)
                    assert abs(G[a * d + k] - 0.7 * acc) < 1e-14 * (1 + abs(acc))
        mom = (m[:, None] * G.reshape(n, d)).sum(0)
        assert np.max(np.abs(mom)) < 1e-13


def test_fpu_beta_force_and_energy_by_hand(orc):
    """The FPU-beta chain written out by hand, independently of the oracle's
    own energy: V(s) = s^2/2 + beta s^4/4 per bond, V'(s) = s + beta s^3, fixed
    ends q_0 = q_{n+1} = 0.
    One site between the ends: both bonds pull it back, g = -2 (q + beta q^3).
    Two sites with bond stiffnesses (1, 3, 1/2), masses (2, 4), beta = 2 at
    q = (1/2, -1/4): bond stretches s = (1/2, -3/4, 1/4), V'(s) = (3/4, -51/32,
    9/32), so g_1 = (3 (-51/32) - 3/4) / 2 = -177/64 and g_2 = ((1/2)(9/32) -
    3 (-51/32)) / 4 = 315/256; U = 1/8 + 1/32 + 3 (9/32 + 81/512) + (1/2)(1/32 +
    1/512) = 1527/1024.  Every value is a dyadic rational, exact in binary64."""
    for beta in (0.0, 0.5, 1.0, 3.0):
        sp = orc.Spec(orc.CHAIN, 1, 1, beta=beta)
        for q in (0.1, -0.37, 1.25):
            with mpmath.workdps(40):
                want = -2 * (mpmath.mpf(q) + mpmath.mpf(beta) * mpmath.mpf(q) ** 3)
            got = orc.force(sp, np.array([q]))[0]
            assert abs(got - want) <= 2e-16 * abs(want), (beta, q)
    sp = orc.Spec(orc.CHAIN, 2, 1, mass=np.array([2.0, 4.0]),
                  coupling=np.array([1.0, 3.0, 0.5]), beta=2.0)
    q = np.array([0.5, -0.25])
    assert np.array_equal(orc.force(sp, q), [-177 / 64, 315 / 256])
    assert orc.energy(sp, q, np.zeros(2)) == 1527 / 1024
    assert orc.energy(sp, q, np.array([1.0, 2.0])) == 1527 / 1024 + 1 / 4 + 1 / 2


def test_forces_are_minus_gradient(orc):
    rng = np.random.default_rng(4)
    cases = [
        orc.Spec(orc.GRAVITY, 4, 3, mass=rng.uniform(0.5, 1.5, 4), G=1.0, eps=0.1),
        orc.Spec(orc.CHAIN, 9, 1, mass=rng.uniform(0.5, 2.0, 9),
                 coupling=rng.uniform(0.5, 2.0, 10), beta=1.3),
        orc.Spec(orc.KEPLER, 1, 3, G=2.0),
        orc.Spec(orc.HENON, 1, 2),
        orc.Spec(orc.HENON_T, 1, 2, G=0.7, beta=0.4),  # energy and force at t = 0
        orc.Spec(orc.DRIVEN, 1, 3, G=-1.3),
    ]
    for sp in cases:
        Q = rng.standard_normal(sp.Dq) * 0.5 + (1.5 if sp.kind == orc.KEPLER else 0.0)
        G = orc.force(sp, Q)
        m = sp.masses_per_component()
        zero = np.zeros(sp.Dq)
        for l in range(sp.Dq):
            e = 1e-5
            qp, qm = Q.copy(), Q.copy()
            qp[l] += e
            qm[l] -= e
            dU = (orc.energy(sp, qp, zero) - orc.energy(sp, qm, zero)) / (2 * e)
            assert abs(G[l] + dU / m[l]) < 1e-7 * (1 + abs(G[l])), (sp.kind, l)


# ---------------------------------------------------------------- time-dependent forces

def test_nonautonomous_henon_reduces_to_classic(orc):
    """Section 3.3's system is the classic Henon-Heiles one for lambda = 1,
    xi = 0: identical trajectories and iteration counts, bit for bit."""
    q0, p0, h, n = [0.0, 0.3], [0.23380903889000242556, 0.2], 2 * np.pi / 64, 2000
    a = orc.integrate(orc.Spec(orc.HENON, 1, 2), q0, p0, h, n, stride=50, want_iters=True)
    b = orc.integrate(orc.Spec(orc.HENON_T, 1, 2, G=1.0, beta=0.0), q0, p0, h, n, stride=50,
                      want_iters=True)
    assert np.array_equal(a["q"], b["q"]) and np.array_equal(a["p"], b["p"])
    assert np.array_equal(a["iters"], b["iters"])


def test_henon_coupling_scaling_is_exact(orc):
    """U_lambda(q) = |q|^2/2 + lambda (q1^2 q2 - q2^3/3) satisfies
    U_lambda(q / lambda) = U_1(q) / lambda^2, so the lambda = 2 orbit from
    (q0/2, p0/2) is the lambda = 1 orbit scaled by 1/2; with a power-of-two
    factor every rounding scales too, so the match is exact."""
    q0, p0, h, n = np.array([0.05, 0.3]), np.array([0.2, 0.2]), 0.2, 1500
    one = orc.integrate(orc.Spec(orc.HENON_T, 1, 2, G=1.0), q0, p0, h, n, stride=25,
                        want_iters=True)
    two = orc.integrate(orc.Spec(orc.HENON_T, 1, 2, G=2.0), q0 / 2, p0 / 2, h, n, stride=25,
                        want_iters=True)
    assert np.array_equal(two["q"] * 2, one["q"]) and np.array_equal(two["p"] * 2, one["p"])
    assert np.array_equal(one["iters"], two["iters"])


@pytest.mark.parametrize("h", [0.5, -0.25])
def test_driven_particle_follows_closed_form(orc, h):
    """q'' = G cos t from t = 0: q = q0 + v0 t + G (1 - cos t), v = v0 + G sin t.
    The stages are evaluated at t_{n-1} + c_i h (eq. IRK_FP), so each step is
    the 8-point Gauss rule for the integral of cos: exact to rounding here;
    evaluating at any other time is off by O(h)."""
    G, n = 1.7, 400
    sp = orc.Spec(orc.DRIVEN, 1, 2, G=G)
    q0, v0 = np.array([0.5, -1.0]), np.array([0.25, 0.0])
    r = orc.integrate(sp, q0, v0, h, n, stride=10, want_iters=True)
    t = (np.arange(n // 10 + 1) * 10 * h)[:, None]
    np.testing.assert_allclose(r["q"], q0 + v0 * t + G * (1 - np.cos(t)), rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["p"], v0 + G * np.sin(t), rtol=0, atol=1e-13)
    assert r["iters"].max() <= 2  # g does not depend on q: exact after one iteration


def test_nonautonomous_henon_energy_balance(orc):
    """For H(q, p, t) = |p|^2/2 + |q|^2/2 + a(t) W(q), a = lambda + xi sin t,
    W = q1^2 q2 - q2^3/3: dH/dt = xi cos(t) W(q(t)) along the orbit.  The
    energy change over the run matches the time integral of the right side
    (Simpson's rule on every-step frames)."""
    lam, xi, h, n = 1.0, 0.3, 0.01, 4000
    sp = orc.Spec(orc.HENON_T, 1, 2, G=lam, beta=xi)
    r = orc.integrate(sp, [0.1, 0.2], [0.15, -0.1], h, n, stride=1)
    q, p = r["q"], r["p"]
    t = np.arange(n + 1) * h
    W = q[:, 0] ** 2 * q[:, 1] - q[:, 1] ** 3 / 3
    H = 0.5 * (p ** 2).sum(1) + 0.5 * (q ** 2).sum(1) + (lam + xi * np.sin(t)) * W
    f = xi * np.cos(t) * W
    integral = h / 3 * (f[0] + f[-1] + 4 * f[1:-1:2].sum() + 2 * f[2:-1:2].sum())
    change = H[-1] - H[0]
    assert abs(change) > 1e-4                 # the forcing does work
    assert abs(change - integral) < 1e-9 * abs(change) + 1e-13


# ---------------------------------------------------------------- building blocks

def test_stopping_rule_sequences(orc):
    def run(deltas):
        mind, prev = np.inf, np.inf
        for k, dl in enumerate(deltas, 1):
            ok, mind, prev = orc.stop_component(dl, mind, prev)
            if ok:
                return k
        return None
    assert run([1e-3, 1e-7, 1e-11, 1e-15, 0.0]) == 5          # exact fixed point
    assert run([1e-3, 1e-7, 2e-16, 1e-16, 3e-16, 2e-16]) == 6  # stagnation: min(D1..D4)<=min(D5,D6)
    assert run([1e-3, 1e-3, 1e-3]) == 3                        # D1 <= min(D2, D3)
    assert run([0.0]) == 1
    assert run([1e-3, 1e-4]) is None                           # history needs k >= 3
    assert run([5.0, 4.0, 3.0, 2.0, 1.0, 0.5]) is None         # still contracting


def test_two_double_add_is_exact(orc):
    rng = np.random.default_rng(9)
    for _ in range(2000):
        hi = rng.standard_normal() * 10.0 ** rng.integers(-3, 4)
        lo = float(np.spacing(abs(hi)) * rng.uniform(-0.5, 0.5))
        lo = float(np.float64(hi + lo) - hi) if hi + lo != hi else lo
        d = rng.standard_normal() * 10.0 ** rng.integers(-12, 0)
        nh, nl = orc.dw_add(hi, lo, d)
        err = Fraction(nh) + Fraction(nl) - (Fraction(hi) + Fraction(lo) + Fraction(d))
        assert abs(err) <= Fraction(np.spacing(abs(nh))) * Fraction(1, 2 ** 50)
        assert nh + nl == nh


def test_numpy_reimplementation_agrees_bitwise(orc):
    tab = orc.tableau()
    sp = orc.Spec(orc.HENON, 1, 2)

    def g(Q):
        return np.stack([-Q[:, 0] - 2 * Q[:, 0] * Q[:, 1],
                         -Q[:, 1] - (Q[:, 0] * Q[:, 0] - Q[:, 1] * Q[:, 1])], axis=1)
    q, v, it = orc.integrate_py(g, [0.0, 0.3], [0.2338, 0.2], 0.3, 60, tab)
    r = orc.integrate(sp, [0.0, 0.3], [0.2338, 0.2], 0.3, 60, stride=60, want_iters=True)
    assert np.array_equal(q, r["q"][-1]) and np.array_equal(v, r["p"][-1])
    assert np.array_equal(it, r["iters"])


# ---------------------------------------------------------------- failure handling

def test_failure_modes(orc):
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    bad = orc.integrate(sp, [0.4, 0.0], [0.0, 2.0], KEP_H, 10, stride=3)
    assert bad["rc"] == orc.EINVAL
    # iteration cap reached before the stopping rule fires: warning, state still written
    r = orc.integrate(sp, [0.4, 0.0], [0.0, 2.0], KEP_H, 5, max_iter=2, want_iters=True)
    assert r["rc"] == orc.ENOCONV and r["stats"]["nonconverged"] == 5
    assert np.all(np.isfinite(r["q"]))
    # a diverging iteration (h w >> 1) is stopped by the stagnation clause of the
    # rule itself (Delta grows, so min(Delta[1..k-2]) <= min(Delta[k-1], Delta[k]))
    r = orc.integrate(orc.Spec(orc.HARMONIC, 1, 1, G=1.0), [1.0], [0.0], 40.0, 1,
                      want_iters=True)
    assert r["iters"][0] == 3
    # coincident bodies without softening: non-finite, remaining frames NaN
    m = np.array([1.0, 1.0])
    g = orc.Spec(orc.GRAVITY, 2, 3, mass=m, G=1.0, eps=0.0)
    r = orc.integrate(g, np.zeros(6), np.zeros(6), 0.1, 4, stride=1)
    assert r["rc"] == orc.ENONFINITE
    assert np.all(np.isnan(r["q"][1:]))
    # batch isolation: the bad instance does not disturb a good one
    good = orc.Spec(orc.GRAVITY, 2, 3, mass=m, G=1.0, eps=0.0)
    q0 = np.concatenate([np.zeros(6), [1.0, 0, 0, -1.0, 0, 0]])
    p0 = np.concatenate([np.zeros(6), [0, 0.5, 0, 0, -0.5, 0]])
    rb = orc.integrate_batch([g, good], q0, p0, 0.1, 4, 4)
    alone = orc.integrate(good, q0[6:], p0[6:], 0.1, 4, stride=4)
    assert rb["status"][0] == orc.ENONFINITE and rb["status"][1] == 0
    np.testing.assert_array_equal(rb["q"][12:], alone["q"].ravel())

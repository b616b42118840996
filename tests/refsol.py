"""Closed-form reference solutions used to pin the oracle (test helpers).

* Kepler's problem q'' = -q/|q|^3 started at a perihelion, solved through
  Kepler's equation M = E - e sin E in multiprecision.
* The exact one-step map of an s-stage Gauss collocation method on the linear
  oscillator q'' = -w^2 q: the [s/s] Pade approximant R(z) = P(z)/P(-z) of
  exp(z), P(z) = sum_k (2s-k)! s! / ((2s)! k! (s-k)!) z^k, applied to the
  first-order system matrix (textbook property of Gauss methods).
"""
from math import factorial

import mpmath


def kepler_perihelion(x0, v0, t, dps=40):
    """Position and velocity at time t for q(0) = (x0, 0), v(0) = (0, v0), mu = 1.

    The orbit elements are derived from the given binary64 initial values
    themselves, so the reference is exact for those inputs.
    """
    with mpmath.workdps(dps):
        x0 = mpmath.mpf(x0)
        v0 = mpmath.mpf(v0)
        a = 1 / (2 / x0 - v0 * v0)
        e = 1 - x0 / a
        n = a ** mpmath.mpf(-1.5)
        M = (n * mpmath.mpf(t)) % (2 * mpmath.pi)
        E = M
        for _ in range(200):
            dE = (E - e * mpmath.sin(E) - M) / (1 - e * mpmath.cos(E))
            E -= dE
            if abs(dE) < mpmath.mpf(10) ** (-(dps - 2)):
                break
        b = a * mpmath.sqrt(1 - e * e)
        Edot = n / (1 - e * mpmath.cos(E))
        q = [a * (mpmath.cos(E) - e), b * mpmath.sin(E)]
        v = [-a * mpmath.sin(E) * Edot, b * mpmath.cos(E) * Edot]
        return q, v


def gauss_pade_map(w2, h, s=8, dps=50):
    """2x2 matrix of one Gauss-collocation step for q'' = -w2 q on (q, v)."""
    with mpmath.workdps(dps):
        p = [mpmath.mpf(factorial(2 * s - k) * factorial(s)) /
             (factorial(2 * s) * factorial(k) * factorial(s - k)) for k in range(s + 1)]
        M = mpmath.matrix([[0, 1], [-mpmath.mpf(w2), 0]]) * mpmath.mpf(h)

        def P(X):
            acc = mpmath.zeros(2)
            pw = mpmath.eye(2)
            for k in range(s + 1):
                acc += p[k] * pw
                pw = pw * X
            return acc
        return P(M) * P(-M) ** -1


def pade_trajectory(w2, h, q0, v0, n, dps=50):
    with mpmath.workdps(dps):
        R = gauss_pade_map(w2, h, dps=dps)
        y = mpmath.matrix([mpmath.mpf(q0), mpmath.mpf(v0)])
        Rn = R ** n
        y = Rn * y
        return y[0], y[1]

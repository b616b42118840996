"""Seeded synthetic inputs for the integrator (no integrator arithmetic here).

These generators are the only code shared by the GPU library's tests and the
CPU oracle's tests: they produce initial states, masses and step sizes and
nothing else.  Every instance draws from its own ``SeedSequence`` child, so an
instance is the same whether it is generated alone or inside a large batch.

Workloads (shapes of the paper's section 5.1 problems and of the synthetic
stand-ins used for throughput):

* :func:`kepler_c1` -- planar Kepler problem, a = 1, e = 0.6, started at the
  perihelion.
* :func:`planetary_systems` -- a central unit mass plus light planets on
  near-circular, near-coplanar orbits (the shape of the outer Solar System
  problem of section 5.1.2, whose ephemeris initial data are not used).
* :func:`plummer` -- an equal-mass Plummer sphere in N-body units (G = M = 1,
  E = -1/4), sampled by the Aarseth-Henon-Wielen (1974) method.
* :func:`fpu_chain` -- a Fermi-Pasta-Ulam-beta chain with fixed ends, energy
  in the lowest mode plus small Gaussian noise.
* :func:`uneven_mix` -- the mixed batch of gravitational systems and chains.
* :func:`schwarzschild_ensemble` -- states of the charged particle near a
  Schwarzschild black hole of section 5.1.1 (theta = pi/2, p_r = 0, r around
  the paper's r = 11, p_theta from H = -1/2).
* :func:`henon_heiles_ensemble` -- Henon-Heiles initial states on the
  surface q1 = 0 (section 5.1.2's problem: q2 = 0.3, p2 = 0.2, H = 1/12 and
  perturbations of it, or other energies).
* :func:`poisson_requests` -- an open-loop Poisson request stream.
"""
from __future__ import annotations

import math

import numpy as np

KEPLER, GRAVITY, CHAIN = 0, 1, 2
BASE_SEED = 20251103


def rng_children(seed, n):
    """One independent Generator per instance."""
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def kepler_c1():
    return dict(kind=KEPLER, n=1, d=2, mass=None, G=1.0, eps=0.0, beta=0.0,
                q=np.array([0.4, 0.0]), p=np.array([0.0, 2.0]), h=2 * math.pi / 128,
                nsteps=10_000)


def _solve_kepler(M, e):
    E = M + e * np.sin(M)
    for _ in range(50):
        E = E - (E - e * np.sin(E) - M) / (1 - e * np.cos(E))
    return E


def _elements_to_cartesian(mu, a, e, inc, Om, om, M):
    """Heliocentric Keplerian elements -> position and velocity (vectorised)."""
    E = _solve_kepler(M, e)
    cE, sE = np.cos(E), np.sin(E)
    b = a * np.sqrt(1 - e * e)
    x, y = a * (cE - e), b * sE
    n = np.sqrt(mu / a ** 3)
    Edot = n / (1 - e * cE)
    vx, vy = -a * sE * Edot, b * cE * Edot
    cO, sO, co, so, ci, si = np.cos(Om), np.sin(Om), np.cos(om), np.sin(om), np.cos(inc), np.sin(inc)
    R = np.stack([
        np.stack([cO * co - sO * so * ci, -cO * so - sO * co * ci], -1),
        np.stack([sO * co + cO * so * ci, -sO * so + cO * co * ci], -1),
        np.stack([so * si, co * si], -1)], -2)  # (..., 3, 2)
    r = np.einsum("...ij,...j->...i", R, np.stack([x, y], -1))
    v = np.einsum("...ij,...j->...i", R, np.stack([vx, vy], -1))
    return r, v


def planetary_systems(n_inst, n_bodies=6, seed=BASE_SEED + 2, m_range=(1e-9, 1e-3),
                      a_range=(5.0, 30.0), e_max=0.05, inc_max_deg=2.0, G=1.0):
    """Central mass 1 plus ``n_bodies - 1`` planets; barycentre at rest at the origin.

    Masses ~ U(m_range); semi-major axes log-uniform in a_range; e ~ U(0, e_max);
    inclination ~ U(0, inc_max); node, perihelion and mean anomaly ~ U(0, 2 pi).
    Returns a list of dicts with q, p (n_bodies * 3 values) and mass.
    """
    k = n_bodies - 1
    draws = np.empty((n_inst, k, 7))
    for i, g in enumerate(rng_children(seed, n_inst)):
        draws[i, :, 0] = g.uniform(*m_range, size=k)
        draws[i, :, 1] = np.exp(g.uniform(math.log(a_range[0]), math.log(a_range[1]), size=k))
        draws[i, :, 2] = g.uniform(0.0, e_max, size=k)
        draws[i, :, 3] = g.uniform(0.0, math.radians(inc_max_deg), size=k)
        draws[i, :, 4:7] = g.uniform(0.0, 2 * math.pi, size=(k, 3))
    m = draws[..., 0]
    r, v = _elements_to_cartesian(G * (1.0 + m), draws[..., 1], draws[..., 2], draws[..., 3],
                                  draws[..., 4], draws[..., 5], draws[..., 6])
    mass = np.concatenate([np.ones((n_inst, 1)), m], axis=1)
    pos = np.concatenate([np.zeros((n_inst, 1, 3)), r], axis=1)
    vel = np.concatenate([np.zeros((n_inst, 1, 3)), v], axis=1)
    mt = mass.sum(1, keepdims=True)[..., None]
    pos -= (mass[..., None] * pos).sum(1, keepdims=True) / mt
    vel -= (mass[..., None] * vel).sum(1, keepdims=True) / mt
    mom = mass[..., None] * vel
    out = []
    for i in range(n_inst):
        out.append(dict(kind=GRAVITY, n=n_bodies, d=3, mass=mass[i].copy(), G=G, eps=0.0, beta=0.0,
                        q=pos[i].ravel().copy(), p=mom[i].ravel().copy(),
                        a_min=float(draws[i, :, 1].min())))
    return out


def planetary_arrays(n_inst, n_bodies=6, seed=BASE_SEED + 2):
    """Packed arrays (mass[n_inst, N], q[n_inst, 3N], p[n_inst, 3N]) of planetary_systems."""
    sy = planetary_systems(n_inst, n_bodies, seed)
    return (np.stack([s["mass"] for s in sy]), np.stack([s["q"] for s in sy]),
            np.stack([s["p"] for s in sy]))


def plummer(n, seed=BASE_SEED + 3, eps=1e-2, r_cut=None):
    """Plummer sphere with n equal masses 1/n in N-body units (G = M = 1, E = -1/4).

    Aarseth, Henon & Wielen (1974): radii from the cumulative mass profile,
    speeds by rejection from g(x) = x^2 (1 - x^2)^(7/2) in units of the local
    escape speed, isotropic directions; then scaled from the Plummer scale
    length 1 to N-body units and recentred.
    """
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    m = np.full(n, 1.0 / n)
    pos = np.empty((n, 3))
    vel = np.empty((n, 3))
    r_cut = 22.8 if r_cut is None else r_cut
    for i in range(n):
        while True:
            X = g.uniform(0.0, 1.0)
            if X <= 0.0:
                continue
            r = (X ** (-2.0 / 3.0) - 1.0) ** -0.5
            if r < r_cut:
                break
        ct = g.uniform(-1.0, 1.0)
        ph = g.uniform(0.0, 2 * math.pi)
        st = math.sqrt(1 - ct * ct)
        pos[i] = r * np.array([st * math.cos(ph), st * math.sin(ph), ct])
        while True:
            x = g.uniform(0.0, 1.0)
            y = g.uniform(0.0, 0.1)
            if y <= x * x * (1 - x * x) ** 3.5:
                break
        ve = math.sqrt(2.0) * (1.0 + r * r) ** -0.25
        ct = g.uniform(-1.0, 1.0)
        ph = g.uniform(0.0, 2 * math.pi)
        st = math.sqrt(1 - ct * ct)
        vel[i] = x * ve * np.array([st * math.cos(ph), st * math.sin(ph), ct])
    pos *= 3 * math.pi / 16
    vel *= math.sqrt(16 / (3 * math.pi))
    pos -= pos.mean(0)
    vel -= vel.mean(0)
    return dict(kind=GRAVITY, n=n, d=3, mass=m, G=1.0, eps=eps, beta=0.0,
                q=pos.ravel(), p=(m[:, None] * vel).ravel(), h=1e-3, nsteps=1000)


def _chain_energy(q, p, beta):
    s = np.diff(np.concatenate([[0.0], q, [0.0]]))
    return 0.5 * np.sum(p * p) + np.sum(0.5 * s * s + 0.25 * beta * s ** 4)


def fpu_chain(n, seed=BASE_SEED + 4, beta=1.0, energy_density=0.01, noise=1e-6, g=None):
    """FPU-beta chain, fixed ends, unit masses and couplings.

    Lowest mode q_i = A sin(pi i / (n+1)), p = 0, with A chosen so that E/n equals
    ``energy_density``; then N(0, noise^2) is added to every q and p.  The step
    is h = U(0.05, 1) x 0.5 / w_max with w_max = 2 sqrt(1 + 3 beta s_max^2).
    """
    g = g or np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    i = np.arange(1, n + 1)
    shape = np.sin(np.pi * i / (n + 1))
    target = energy_density * n
    lo, hi = 0.0, 10.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _chain_energy(mid * shape, np.zeros(n), beta) < target:
            lo = mid
        else:
            hi = mid
    q = lo * shape + noise * g.standard_normal(n)
    p = noise * g.standard_normal(n)
    s_max = float(np.max(np.abs(np.diff(np.concatenate([[0.0], q, [0.0]])))))
    scale = 0.5 / (2.0 * math.sqrt(1.0 + 3.0 * beta * s_max ** 2))
    h = g.uniform(0.05, 1.0) * scale
    return dict(kind=CHAIN, n=n, d=1, mass=None, G=1.0, eps=0.0, beta=beta, q=q, p=p, h=h)


def _max_pair_frequency(inst):
    q = inst["q"].reshape(-1, 3)
    m = inst["mass"]
    d = q[:, None, :] - q[None, :, :]
    r = np.sqrt(np.sum(d * d, -1))
    iu = np.triu_indices(len(m), 1)
    return float(np.max(np.sqrt(inst["G"] * (m[:, None] + m[None, :])[iu] / r[iu] ** 3)))


MIX_CLASSES = [("gravity", 3), ("gravity", 6), ("gravity", 16), ("gravity", 64),
               ("chain", 32), ("chain", 256), ("chain", 1024)]


def uneven_mix(n_inst=4096, seed=BASE_SEED + 4, steps_range=(1e3, 1e5), classes=None,
               step_multiple=100):
    """The uneven batch: classes uniform over MIX_CLASSES, per-instance h and steps.

    Gravity systems are generated as planetary_systems with the class's body
    count; their step is h = U(0.05, 1) x 0.5 / w_max with w_max the fastest
    pairwise frequency max_{a<b} sqrt(G (m_a + m_b) / r_ab^3) of the initial
    configuration (star-planet and planet-planet pairs alike).  Steps are
    log-uniform in steps_range, rounded to a multiple of step_multiple (so an
    output frame can fall on step 1000 of every instance).
    """
    classes = classes or MIX_CLASSES
    out = []
    for i, g in enumerate(rng_children(seed, n_inst)):
        kind, size = classes[int(g.integers(len(classes)))]
        sub = int(g.integers(2 ** 62))
        if kind == "gravity":
            inst = planetary_systems(1, n_bodies=size, seed=sub)[0]
            inst["h"] = float(g.uniform(0.05, 1.0) * 0.5 / _max_pair_frequency(inst))
        else:
            inst = fpu_chain(size, seed=sub)
        steps = math.exp(g.uniform(math.log(steps_range[0]), math.log(steps_range[1])))
        inst["nsteps"] = max(step_multiple, int(round(steps / step_multiple)) * step_multiple)
        inst["cls"] = f"{kind}{size}"
        out.append(inst)
    return out


def poisson_requests(rate, n_req, seed=BASE_SEED + 5, steps_range=(1e3, 1e6), stride=100,
                     plummer_sizes=(64, 128, 256, 512)):
    """Open-loop Poisson stream: (arrival_time_s, instance) pairs.

    Each request is drawn from the uneven mix or is a Plummer cluster with N from
    plummer_sizes; steps log-uniform in steps_range rounded to a multiple of
    stride (the output period).
    """
    g = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    t = np.cumsum(g.exponential(1.0 / rate, size=n_req))
    out = []
    n_cls = len(MIX_CLASSES) + 1
    for k in range(n_req):
        c = int(g.integers(n_cls))
        sub = int(g.integers(2 ** 62))
        if c < len(MIX_CLASSES):
            inst = uneven_mix(1, seed=sub, classes=[MIX_CLASSES[c]])[0]
        else:
            n = int(plummer_sizes[int(g.integers(len(plummer_sizes)))])
            inst = plummer(n, seed=sub)
            inst["cls"] = f"plummer{n}"
        steps = math.exp(g.uniform(math.log(steps_range[0]), math.log(steps_range[1])))
        inst["nsteps"] = max(stride, int(round(steps / stride)) * stride)
        inst["stride"] = stride
        out.append((float(t[k]), inst))
    return out


def henon_heiles_ensemble(n, seed=BASE_SEED + 6, energy=1 / 12, q2_range=(0.25, 0.35),
                          p2_range=(0.15, 0.25)):
    """n Henon-Heiles states (q of shape (n, 2), p of shape (n, 2)): q1 = 0,
    q2 and p2 uniform in the given ranges, p1 > 0 from the energy (a number,
    or a (lo, hi) range to draw from), with
    H = (p1^2 + p2^2)/2 + (q1^2 + q2^2)/2 + q1^2 q2 - q2^3/3.
    The defaults surround the paper's regular orbit (q2 = 0.3, p2 = 0.2,
    H = 1/12)."""
    rng = np.random.default_rng(seed)
    q, p = [], []
    while len(q) < n:
        E = rng.uniform(*energy) if np.ndim(energy) else float(energy)
        q2 = rng.uniform(*q2_range)
        p2 = rng.uniform(*p2_range)
        rest = 2 * E - p2 ** 2 - q2 ** 2 + 2.0 / 3.0 * q2 ** 3
        if rest <= 0:
            continue
        q.append([0.0, q2])
        p.append([np.sqrt(rest), p2])
    return np.array(q), np.array(p)


SBH_PARAMS = (0.995, 4.6, 8.9e-4)  # E, L, beta of section 5.1.1


def schwarzschild_ensemble(n, seed=BASE_SEED + 7, r_range=(10.5, 11.5), params=SBH_PARAMS,
                           energy=-0.5):
    """n states y = (r, theta, p_r, p_theta) of eq. Ham_SBH: theta = pi/2,
    p_r = 0, r uniform in r_range, p_theta > 0 from H = energy (the paper:
    r = 11, H = -1/2)."""
    E, L, b = params
    rng = np.random.default_rng(seed)
    r0 = rng.uniform(r_range[0], r_range[1], n)
    A = 1 - 2 / r0
    w = L - b * r0 * r0 / 2
    pth2 = 2 * r0 * r0 * (energy + E * E / (2 * A) - w * w / (2 * r0 * r0))
    if np.any(pth2 <= 0):
        raise ValueError("no p_theta > 0 reaches the requested energy for some r")
    return np.stack([r0, np.full(n, np.pi / 2), np.zeros(n), np.sqrt(pth2)], 1)

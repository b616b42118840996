"""Python access to the CPU oracle (FP64 and double-double).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  Nothing here is shared
with the GPU library.

* :func:`build` compiles ``irkgl16_oracle.c`` and ``irkgl16_dd.c`` with gcc in
  strict IEEE mode (``-O2 -ffp-contract=off``, no fast-math) into
  ``oracle/liborc.so``.
* :func:`integrate` / :func:`integrate_batch` / :func:`integrate_dd` wrap the
  C entry points with numpy arrays.
* :func:`integrate_py` is a second, independent FP64 implementation written
  with numpy in the paper's s-vector notation (section 2.5): rows of an
  (8, Dq) array are stages.  It is only used on small cases to cross-check
  the C oracle.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IRKGL16_ORACLE_LIB names a prebuilt copy to load instead (the CPU tests'
# sanitizer build); it is loaded as given, never rebuilt.
LIB_OVERRIDE = os.environ.get("IRKGL16_ORACLE_LIB")
LIB_PATH = LIB_OVERRIDE or os.path.join(HERE, "liborc.so")
SOURCES = ["irkgl16_oracle.c", "irkgl16_dd.c", "irkgl16_ode.c", "irkgl16_split.c"]

KEPLER, GRAVITY, CHAIN, HARMONIC, CONST, HENON = 0, 1, 2, 10, 11, 12
HENON_T, DRIVEN = 13, 14  # time-dependent: lambda = G, xi = beta; g = G cos t
# first-order problems y' = f(t, y) (irkgl16_ode.c): D = n * d
ODE_OSC, ODE_KEPLER, ODE_DAMPED, ODE_SBH, ODE_DRIVEN = 20, 21, 22, 23, 24
# explicit splitting baselines (irkgl16_split.c)
STRANG, SUZ90 = 1, 2
FLAG_NO_COMPENSATION, FLAG_NAIVE_ETA, FLAG_NO_EXTRAPOLATION = 1, 2, 4
OK, EINVAL, ENOMEM, ENONFINITE, ENOCONV = 0, -1, -2, -4, 1


def build(force=True, out=None, extra_flags=()):
    """Compile the oracle shared library (gcc, strict IEEE binary64).
    extra_flags: added options (the sanitizer build of the CPU tests)."""
    out = out or os.path.join(HERE, "liborc.so")
    if not force and os.path.exists(out):
        return out
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas", *extra_flags, "-o", tmp] + srcs + \
          ["-lm"]
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, out)
    return out


class Problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("d", C.c_int32),
                ("mass", C.POINTER(C.c_double)), ("coupling", C.POINTER(C.c_double)),
                ("G", C.c_double), ("eps", C.c_double), ("beta", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("steps_done", C.c_int64), ("iterations", C.c_int64), ("max_k", C.c_int32),
                ("nonconverged", C.c_int32), ("status", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        srcs = [os.path.join(HERE, s) for s in SOURCES] + [os.path.join(HERE, "tableau.h")]
        if not LIB_OVERRIDE and (not os.path.exists(LIB_PATH) or any(
                os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in srcs)):
            build()
        L = C.CDLL(LIB_PATH)
        dp, i64p, i32p = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.orc_integrate.argtypes = [C.POINTER(Problem), dp, dp, C.c_double, C.c_int64, C.c_int64,
                                    C.c_int32, C.c_int32, dp, dp, i32p, dp, C.POINTER(Stats)]
        L.orc_integrate.restype = C.c_int
        L.orc_integrate_batch.argtypes = [C.c_int32, C.POINTER(Problem), dp, dp, dp, i64p, i64p,
                                          C.c_int32, C.c_int32, dp, dp, i64p, i32p]
        L.orc_integrate_batch.restype = C.c_int
        L.orc_force.argtypes = [C.POINTER(Problem), dp, dp]
        L.orc_force.restype = None
        L.orc_force_t.argtypes = [C.POINTER(Problem), dp, dp, C.c_double]
        L.orc_force_t.restype = None
        L.orc_energy.argtypes = [C.POINTER(Problem), dp, dp]
        L.orc_energy.restype = C.c_double
        L.orc_dw_add.argtypes = [dp, dp, C.c_double]
        L.orc_dw_add.restype = None
        L.orc_stop_component.argtypes = [C.c_double, dp, dp]
        L.orc_stop_component.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_tableau.argtypes = [dp] * 5
        L.orc_tableau.restype = None
        L.ddo_integrate.argtypes = [C.POINTER(Problem), dp, dp, C.c_double, C.c_int64, C.c_int64,
                                    C.c_int32, dp, dp, dp, dp, i32p]
        L.ddo_integrate.restype = C.c_int
        L.ddo_energy.argtypes = [C.POINTER(Problem), dp, dp, dp, dp, dp, dp]
        L.ddo_energy.restype = None
        L.orc_rhs.argtypes = [C.POINTER(Problem), C.c_double, dp, dp]
        L.orc_rhs.restype = None
        L.orc_energy_ode.argtypes = [C.POINTER(Problem), dp]
        L.orc_energy_ode.restype = C.c_double
        L.orc_integrate_ode.argtypes = [C.POINTER(Problem), dp, C.c_double, C.c_int64, C.c_int64,
                                        C.c_int32, dp, i32p, C.POINTER(Stats)]
        L.orc_integrate_ode.restype = C.c_int
        L.orc_integrate_ode_batch.argtypes = [C.c_int32, C.POINTER(Problem), dp, dp, i64p, i64p,
                                              C.c_int32, dp, i64p, i32p]
        L.orc_integrate_ode_batch.restype = C.c_int
        L.orc_integrate_s.argtypes = [C.POINTER(Problem), C.c_int32, dp, dp, C.c_double, C.c_int64,
                                      C.c_int64, C.c_int32, dp, dp, i32p, C.POINTER(Stats)]
        L.orc_integrate_s.restype = C.c_int
        L.orc_integrate_batch_s.argtypes = [C.c_int32, C.c_int32, C.POINTER(Problem), dp, dp, dp,
                                            i64p, i64p, C.c_int32, C.c_int32, dp, dp, i64p, i32p]
        L.orc_integrate_batch_s.restype = C.c_int
        L.orc_integrate_ode_s.argtypes = [C.POINTER(Problem), C.c_int32, dp, C.c_double, C.c_int64,
                                          C.c_int64, C.c_int32, dp, i32p, C.POINTER(Stats)]
        L.orc_integrate_ode_s.restype = C.c_int
        L.orc_integrate_ode_batch_s.argtypes = [C.c_int32, C.c_int32, C.POINTER(Problem), dp, dp,
                                                i64p, i64p, C.c_int32, dp, i64p, i32p]
        L.orc_integrate_ode_batch_s.restype = C.c_int
        L.orc_split_integrate.argtypes = [C.POINTER(Problem), C.c_int32, dp, dp, C.c_double,
                                          C.c_int64, C.c_int64, dp, dp, C.POINTER(Stats)]
        L.orc_split_integrate.restype = C.c_int
        L.orc_split_integrate_batch.argtypes = [C.c_int32, C.c_int32, C.POINTER(Problem), dp, dp,
                                                dp, i64p, i64p, dp, dp, i32p]
        L.orc_split_integrate_batch.restype = C.c_int
        _lib = L
    return _lib


def set_threads(n):
    """Thread count of the oracle's parallel loops (n <= 0: the OpenMP default)."""
    lib().orc_set_threads(int(n))


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Spec:
    """A problem description held alive together with its ctypes struct."""

    def __init__(self, kind, n, d, mass=None, coupling=None, G=1.0, eps=0.0, beta=0.0):
        self.kind, self.n, self.d = int(kind), int(n), int(d)
        self.mass = None if mass is None else np.ascontiguousarray(mass, dtype=np.float64)
        self.coupling = None if coupling is None else np.ascontiguousarray(coupling, np.float64)
        self.G, self.eps, self.beta = float(G), float(eps), float(beta)

    @property
    def Dq(self):
        return self.n * self.d

    def masses_per_component(self):
        if self.kind in (GRAVITY, CHAIN) and self.mass is not None:
            return np.repeat(self.mass, self.d)
        return np.ones(self.Dq)

    def struct(self):
        return Problem(self.kind, self.n, self.d,
                       _dp(self.mass) if self.mass is not None else None,
                       _dp(self.coupling) if self.coupling is not None else None,
                       self.G, self.eps, self.beta)


def integrate(spec, q0, p0, h, nsteps, stride=1, max_iter=100, flags=0, want_iters=False,
              want_delta1=False):
    """FP64 oracle, one instance.  Returns dict(q, p, iters, delta1, stats, rc)."""
    L = lib()
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    nf = nsteps // stride + 1
    qo = np.empty((nf, spec.Dq))
    po = np.empty((nf, spec.Dq))
    it = np.zeros(max(nsteps, 1), np.int32) if want_iters else None
    d1 = np.zeros(max(nsteps, 1)) if want_delta1 else None
    st = Stats()
    pr = spec.struct()
    rc = L.orc_integrate(C.byref(pr), _dp(q0), _dp(p0), float(h), int(nsteps), int(stride),
                         int(max_iter), int(flags), _dp(qo), _dp(po),
                         it.ctypes.data_as(C.POINTER(C.c_int32)) if it is not None else None,
                         _dp(d1) if d1 is not None else None, C.byref(st))
    return dict(q=qo, p=po, iters=None if it is None else it[:nsteps],
                delta1=None if d1 is None else d1[:nsteps],
                stats=dict(steps_done=st.steps_done, iterations=st.iterations, max_k=st.max_k,
                           nonconverged=st.nonconverged, status=st.status), rc=rc)


def integrate_s(spec, s, q0, p0, h, nsteps, stride=1, max_iter=100, want_iters=False):
    """Second-order FP64 oracle with the s-stage member (s = 2, 4, 6, 8)."""
    L = lib()
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    nf = nsteps // stride + 1
    qo = np.empty((nf, spec.Dq))
    po = np.empty((nf, spec.Dq))
    it = np.zeros(max(nsteps, 1), np.int32) if want_iters else None
    st = Stats()
    pr = spec.struct()
    rc = L.orc_integrate_s(C.byref(pr), int(s), _dp(q0), _dp(p0), float(h), int(nsteps),
                           int(stride), int(max_iter), _dp(qo), _dp(po),
                           it.ctypes.data_as(C.POINTER(C.c_int32)) if it is not None else None,
                           C.byref(st))
    return dict(q=qo, p=po, iters=None if it is None else it[:nsteps],
                stats=dict(steps_done=st.steps_done, iterations=st.iterations, max_k=st.max_k,
                           nonconverged=st.nonconverged, status=st.status), rc=rc)


def integrate_batch(specs, q0, p0, h, nsteps, stride, max_iter=100, flags=0, s=8):
    """FP64 oracle over many instances (OpenMP).  Packed arrays as the library;
    s stages (default 8; flags apply to s = 8 only)."""
    L = lib()
    n = len(specs)
    arr = (Problem * n)(*[s.struct() for s in specs])
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    h = np.ascontiguousarray(np.broadcast_to(h, (n,)), np.float64)
    ns = np.ascontiguousarray(np.broadcast_to(nsteps, (n,)), np.int64)
    sd = np.ascontiguousarray(np.broadcast_to(stride, (n,)), np.int64)
    tot = int(sum(s.Dq * (int(a) // int(b) + 1) for s, a, b in zip(specs, ns, sd)))
    qo = np.empty(tot)
    po = np.empty(tot)
    iters = np.zeros(n, np.int64)
    status = np.zeros(n, np.int32)
    rc = L.orc_integrate_batch_s(n, int(s), arr, _dp(q0), _dp(p0), _dp(h),
                                 ns.ctypes.data_as(C.POINTER(C.c_int64)),
                                 sd.ctypes.data_as(C.POINTER(C.c_int64)), int(max_iter),
                                 int(flags), _dp(qo), _dp(po),
                                 iters.ctypes.data_as(C.POINTER(C.c_int64)),
                                 status.ctypes.data_as(C.POINTER(C.c_int32)))
    return dict(q=qo, p=po, iters=iters, status=status, rc=rc)


def integrate_dd(spec, q0, p0, h, nsteps, stride=1, max_iter=200, want_iters=False):
    """Double-double oracle.  Returns dict(q_hi, q_lo, p_hi, p_lo, iters, rc)."""
    L = lib()
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    nf = nsteps // stride + 1
    out = [np.empty((nf, spec.Dq)) for _ in range(4)]
    it = np.zeros(max(nsteps, 1), np.int32) if want_iters else None
    pr = spec.struct()
    rc = L.ddo_integrate(C.byref(pr), _dp(q0), _dp(p0), float(h), int(nsteps), int(stride),
                         int(max_iter), *[_dp(o) for o in out],
                         it.ctypes.data_as(C.POINTER(C.c_int32)) if it is not None else None)
    return dict(q_hi=out[0], q_lo=out[1], p_hi=out[2], p_lo=out[3],
                iters=None if it is None else it[:nsteps], rc=rc)


def force(spec, Q, t=None):
    """g(Q) (or g(Q, t) for the time-dependent kinds)."""
    L = lib()
    Q = np.ascontiguousarray(Q, np.float64)
    G = np.empty_like(Q)
    pr = spec.struct()
    if t is None:
        L.orc_force(C.byref(pr), _dp(Q), _dp(G))
    else:
        L.orc_force_t(C.byref(pr), _dp(Q), _dp(G), float(t))
    return G


def energy(spec, q, p):
    """H(q, p) for one state (binary64)."""
    L = lib()
    q = np.ascontiguousarray(q, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    pr = spec.struct()
    return L.orc_energy(C.byref(pr), _dp(q), _dp(p))


def energy_dd(spec, qh, ql, ph, pl):
    L = lib()
    arrs = [np.ascontiguousarray(a, np.float64) for a in (qh, ql, ph, pl)]
    hh, hl = C.c_double(), C.c_double()
    pr = spec.struct()
    L.ddo_energy(C.byref(pr), *[_dp(a) for a in arrs], C.byref(hh), C.byref(hl))
    return hh.value, hl.value


def tableau():
    """The binary64 tables compiled into the oracle (c, b, eta, mu, nu)."""
    L = lib()
    c, b = np.empty(8), np.empty(8)
    eta, mu, nu = np.empty((8, 8)), np.empty((8, 8)), np.empty((8, 8))
    L.orc_tableau(_dp(c), _dp(b), _dp(eta), _dp(mu), _dp(nu))
    return dict(c=c, b=b, eta=eta, mu=mu, nu=nu)


def dw_add(hi, lo, delta):
    L = lib()
    h, l = C.c_double(hi), C.c_double(lo)
    L.orc_dw_add(C.byref(h), C.byref(l), float(delta))
    return h.value, l.value


def stop_component(delta, mind, prev):
    L = lib()
    m, p = C.c_double(mind), C.c_double(prev)
    ok = L.orc_stop_component(float(delta), C.byref(m), C.byref(p))
    return bool(ok), m.value, p.value


# ---------------------------------------------------------------------------
# Independent numpy version (s-vector notation of section 2.5).
# ---------------------------------------------------------------------------

def integrate_py(g, q0, v0, h, nsteps, tables, max_iter=100):
    """Second FP64 implementation for small cases; returns (q, v, iters).

    ``g`` maps an (8, Dq) array of stage positions to an (8, Dq) array of
    accelerations.  Stage vectors are the rows; the 8x8 contractions are
    written as explicit loops over j in ascending order so that the rounding
    matches a plain left-to-right sum.
    """
    c = np.asarray(tables["c"])
    b = np.asarray(tables["b"])
    eta, mu, nu = (np.asarray(tables[k]) for k in ("eta", "mu", "nu"))
    hb = h * b
    q = np.array(q0, dtype=np.float64)
    v = np.array(v0, dtype=np.float64)
    ql = np.zeros_like(q)
    vl = np.zeros_like(v)
    Dq = q.size
    Rprev = np.zeros((8, Dq))
    iters = []

    def two_sum_update(hi, lo, d):
        s = hi + d
        bb = s - hi
        e = (hi - (s - bb)) + (d - bb)
        t = e + lo
        nh = s + t
        return nh, t - (nh - s)

    for _ in range(nsteps):
        V0 = np.empty((8, Dq))
        for i in range(8):
            acc = np.zeros(Dq)
            for j in range(8):
                acc = acc + nu[i, j] * Rprev[j]
            V0[i] = v + acc
        Q = np.empty((8, Dq))
        for i in range(8):
            acc = np.zeros(Dq)
            for j in range(8):
                acc = acc + mu[i, j] * (hb[j] * V0[j])
            Q[i] = q + acc
        mind = np.full(Dq, np.inf)
        prev = np.full(Dq, np.inf)
        k = 0
        while True:
            k += 1
            R = hb[:, None] * g(Q)
            Qn = np.empty_like(Q)
            for i in range(8):
                acc = np.zeros(Dq)
                for j in range(8):
                    acc = acc + eta[i, j] * R[j]
                Qn[i] = q + h * (c[i] * v + acc)
            delta = np.max(np.abs(Qn - Q), axis=0)
            ok = (delta == 0) | (mind <= np.minimum(prev, delta))
            mind = np.minimum(mind, prev)
            prev = delta
            Q = Qn
            if ok.all() or k >= max_iter:
                break
        iters.append(k)
        sv = np.zeros(Dq)
        sc = np.zeros(Dq)
        for i in range(8):
            sv = sv + R[i]
        for i in range(8):
            sc = sc + c[i] * R[i]
        v, vl = two_sum_update(v, vl, sv)
        q, ql = two_sum_update(q, ql, h * (v - sc))
        Rprev = R
    return q, v, np.array(iters)


# ---------------------------------------------------------------- first-order form

def rhs(spec, t, Y):
    """f(t, Y) of a first-order kind."""
    L = lib()
    Y = np.ascontiguousarray(Y, np.float64)
    F = np.empty_like(Y)
    pr = spec.struct()
    L.orc_rhs(C.byref(pr), float(t), _dp(Y), _dp(F))
    return F


def energy_ode(spec, y):
    L = lib()
    y = np.ascontiguousarray(y, np.float64)
    pr = spec.struct()
    return L.orc_energy_ode(C.byref(pr), _dp(y))


def integrate_ode(spec, y0, h, nsteps, stride=1, max_iter=100, want_iters=False, s=8):
    """First-order (mu form) FP64 oracle, one instance, s stages (default 8).
    Returns dict(y, iters, stats, rc)."""
    L = lib()
    y0 = np.ascontiguousarray(y0, np.float64)
    nf = nsteps // stride + 1
    yo = np.empty((nf, spec.Dq))
    it = np.zeros(max(nsteps, 1), np.int32) if want_iters else None
    st = Stats()
    pr = spec.struct()
    itp = it.ctypes.data_as(C.POINTER(C.c_int32)) if it is not None else None
    if s == 8:
        rc = L.orc_integrate_ode(C.byref(pr), _dp(y0), float(h), int(nsteps), int(stride),
                                 int(max_iter), _dp(yo), itp, C.byref(st))
    else:
        rc = L.orc_integrate_ode_s(C.byref(pr), int(s), _dp(y0), float(h), int(nsteps),
                                   int(stride), int(max_iter), _dp(yo), itp, C.byref(st))
    return dict(y=yo, iters=None if it is None else it[:nsteps],
                stats=dict(steps_done=st.steps_done, iterations=st.iterations, max_k=st.max_k,
                           nonconverged=st.nonconverged, status=st.status), rc=rc)


def integrate_ode_batch(specs, y0, h, nsteps, stride, max_iter=100, s=8):
    """First-order oracle over many instances (OpenMP), packed as the library;
    s stages (default 8)."""
    L = lib()
    n = len(specs)
    arr = (Problem * n)(*[s.struct() for s in specs])
    y0 = np.ascontiguousarray(y0, np.float64)
    h = np.ascontiguousarray(np.broadcast_to(h, (n,)), np.float64)
    ns = np.ascontiguousarray(np.broadcast_to(nsteps, (n,)), np.int64)
    sd = np.ascontiguousarray(np.broadcast_to(stride, (n,)), np.int64)
    tot = int(sum(s.Dq * (int(a) // int(b) + 1) for s, a, b in zip(specs, ns, sd)))
    yo = np.empty(tot)
    iters = np.zeros(n, np.int64)
    status = np.zeros(n, np.int32)
    rc = L.orc_integrate_ode_batch_s(n, int(s), arr, _dp(y0), _dp(h),
                                     ns.ctypes.data_as(C.POINTER(C.c_int64)),
                                     sd.ctypes.data_as(C.POINTER(C.c_int64)), int(max_iter),
                                     _dp(yo), iters.ctypes.data_as(C.POINTER(C.c_int64)),
                                     status.ctypes.data_as(C.POINTER(C.c_int32)))
    return dict(y=yo, iters=iters, status=status, rc=rc)


# ---------------------------------------------------------------- explicit splitting

def split_integrate(spec, method, q0, p0, h, nsteps, stride=1):
    """Explicit symmetric composition (STRANG or SUZ90) in ABA form, one
    instance.  Returns dict(q, p, rc)."""
    L = lib()
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    nf = nsteps // stride + 1
    qo = np.empty((nf, spec.Dq))
    po = np.empty((nf, spec.Dq))
    st = Stats()
    pr = spec.struct()
    rc = L.orc_split_integrate(C.byref(pr), int(method), _dp(q0), _dp(p0), float(h),
                               int(nsteps), int(stride), _dp(qo), _dp(po), C.byref(st))
    return dict(q=qo, p=po, rc=rc, steps_done=st.steps_done)


def split_integrate_batch(specs, method, q0, p0, h, nsteps, stride):
    L = lib()
    n = len(specs)
    arr = (Problem * n)(*[s.struct() for s in specs])
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    h = np.ascontiguousarray(np.broadcast_to(h, (n,)), np.float64)
    ns = np.ascontiguousarray(np.broadcast_to(nsteps, (n,)), np.int64)
    sd = np.ascontiguousarray(np.broadcast_to(stride, (n,)), np.int64)
    tot = int(sum(s.Dq * (int(a) // int(b) + 1) for s, a, b in zip(specs, ns, sd)))
    qo = np.empty(tot)
    po = np.empty(tot)
    status = np.zeros(n, np.int32)
    rc = L.orc_split_integrate_batch(n, int(method), arr, _dp(q0), _dp(p0), _dp(h),
                                     ns.ctypes.data_as(C.POINTER(C.c_int64)),
                                     sd.ctypes.data_as(C.POINTER(C.c_int64)), _dp(qo), _dp(po),
                                     status.ctypes.data_as(C.POINTER(C.c_int32)))
    return dict(q=qo, p=po, status=status, rc=rc)

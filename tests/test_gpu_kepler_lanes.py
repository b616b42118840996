"""Kepler orbits in batches of at most LIMIT run in the one-wavefront-per-
orbit latency kernel; larger batches run in the eight-slot small-system
kernel.  Both evaluate the same operations in the same order, so an orbit's
trajectory, per-step iteration counts and status must not depend on the batch
it comes in: bit-identical results alone, in a batch of LIMIT and in a batch
of BIG, in both arithmetic modes, in 2 and 3 dimensions, across launches
(plain form: one launch per step, the state handed over through device
memory), for a non-finite orbit, at iteration caps, and when served in
slices."""
import math

import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K

pytestmark = pytest.mark.gpu

LIMIT = 8192      # the latency kernel's largest batch (kKeplerLaneMaxBatch)
BIG = LIMIT + 8   # a batch for the eight-slot kernel


def _orbits(n, d, seed):
    """Bound orbits around a unit central mass (G = 1): radius 0.3..1.5,
    speed 0.6..1.3 of the circular speed, random direction of motion in the
    plane normal to a random axis (d = 3)."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(0.3, 1.5, n)
    f = rng.uniform(0.6, 1.3, n)
    if d == 2:
        a = rng.uniform(0, 2 * math.pi, n)
        q = np.stack([r * np.cos(a), r * np.sin(a)], 1)
        t = np.stack([-np.sin(a), np.cos(a)], 1)
    else:
        u = rng.normal(size=(n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        w = rng.normal(size=(n, 3))
        w -= np.sum(w * u, 1, keepdims=True) * u
        w /= np.linalg.norm(w, axis=1, keepdims=True)
        q = r[:, None] * u
        t = w
    p = (f * np.sqrt(1.0 / r))[:, None] * t
    return q.ravel(), p.ravel()


def _run(n, d, q0, p0, steps, stride, flags=0, max_iter=100):
    probs = [dict(kind=K.IRKGL16_KEPLER, n=1, d=d, G=1.0)] * n
    integ = K.Integrator(probs, record_iters=True, flags=flags, max_iter=max_iter)
    return integ.integrate(q0, p0, 2 * math.pi / 128, steps, stride)


def _same(a, b, lo, hi, steps):
    """a (whole result) against instances lo..hi-1 of b."""
    qa, pa, sa, _ = a
    qb, pb, sb, _ = b
    nfq = qa.size // (hi - lo)
    assert np.array_equal(qa, qb[lo * nfq:hi * nfq], equal_nan=True)
    assert np.array_equal(pa, pb[lo * nfq:hi * nfq], equal_nan=True)
    assert np.array_equal(sa["step_iters"], sb["step_iters"][lo * steps:hi * steps])
    assert np.array_equal(sa["inst_iterations"], sb["inst_iterations"][lo:hi])
    assert np.array_equal(sa["inst_status"], sb["inst_status"][lo:hi])


@pytest.mark.parametrize("flags", [0, K.IRKGL16_REPRODUCIBLE])
@pytest.mark.parametrize("d", [2, 3])
def test_orbit_alone_equals_in_batches(flags, d):
    N, steps, stride = BIG, 600, 50
    q0, p0 = _orbits(N, d, seed=50 + d)
    big = _run(N, d, q0, p0, steps, stride, flags)  # eight-slot kernel
    assert big[3] == 0
    few = _run(LIMIT, d, q0[:LIMIT * d], p0[:LIMIT * d], steps, stride, flags)  # latency kernel
    _same(few, big, 0, LIMIT, steps)
    for i in (0, 37, N - 1):
        one = _run(1, d, q0[i * d:(i + 1) * d], p0[i * d:(i + 1) * d], steps, stride, flags)
        _same(one, big, i, i + 1, steps)


@pytest.mark.parametrize("d", [2, 3])
def test_plain_form_equals_batched(d):
    N, steps, stride = BIG, 80, 10
    q0, p0 = _orbits(N, d, seed=7)
    big = _run(N, d, q0, p0, steps, stride)
    probs = [dict(kind=K.IRKGL16_KEPLER, n=1, d=d, G=1.0)] * 3
    integ = K.Integrator(probs, record_iters=True, flags=K.IRKGL16_PLAIN)
    plain = integ.integrate(q0[:3 * d], p0[:3 * d], 2 * math.pi / 128, steps, stride)
    _same(plain, big, 0, 3, steps)


def test_nonfinite_orbit_alone_equals_in_batch():
    """An orbit started at rest at the centre (every stage value at r = 0)
    turns non-finite in its first step: NaN frames, status non-finite, the
    other orbits unaffected."""
    N, d, steps, stride = BIG, 2, 20, 5
    q0, p0 = _orbits(N, d, seed=11)
    q0[3 * d:4 * d] = 0.0
    p0[3 * d:4 * d] = 0.0
    big = _run(N, d, q0, p0, steps, stride)
    few = _run(8, d, q0[:8 * d], p0[:8 * d], steps, stride)
    assert big[3] == K.IRKGL16_ENONFINITE and few[3] == K.IRKGL16_ENONFINITE
    assert few[2]["inst_status"][3] == K.IRKGL16_ENONFINITE
    nf = steps // stride + 1
    assert np.all(np.isnan(few[0][3 * nf * d + d:4 * nf * d]))
    assert np.all(np.isfinite(np.delete(few[0], np.s_[3 * nf * d:4 * nf * d])))
    _same(few, big, 0, 8, steps)


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_iteration_cap_alone_equals_in_batch(cap):
    """Steps cut at 1, 2 or 3 iterations: the caps on either side of the
    iteration where the stopping rule first compares earlier norms."""
    N, d, steps, stride = BIG, 2, 30, 10
    q0, p0 = _orbits(N, d, seed=12)
    big = _run(N, d, q0, p0, steps, stride, max_iter=cap)
    few = _run(5, d, q0[:5 * d], p0[:5 * d], steps, stride, max_iter=cap)
    if cap < 3:
        assert few[3] == K.IRKGL16_ENOCONV
    _same(few, big, 0, 5, steps)


@pytest.mark.parametrize("flags", [0, K.IRKGL16_REPRODUCIBLE])
def test_served_orbits_equal_alone(flags):
    """Served Kepler requests (the latency kernel, resumed slice after slice
    under per-slice step budgets) give the bits of the same orbit alone."""
    from paper_2511_03655_amd import serve
    d, n_req = 3, 6
    q0, p0 = _orbits(n_req, d, seed=21)
    reqs = []
    for i in range(n_req):
        inst = dict(kind=K.IRKGL16_KEPLER, n=1, d=d, mass=None, G=1.0, eps=0.0, beta=0.0,
                    q=q0[i * d:(i + 1) * d].copy(), p=p0[i * d:(i + 1) * d].copy(),
                    h=2 * math.pi / 128, nsteps=300 + 100 * i, stride=50, cls="kepler")
        reqs.append((0.001 * i, inst))
    out = serve.run_stream(reqs, cap_bytes=1 << 26, slice_steps=70, keep_frames=True,
                           flags=flags)
    for (t, inst), (q, p, info, rc) in zip(reqs, out["results"]):
        qa, pa, sa, rca = _run(1, d, inst["q"], inst["p"], inst["nsteps"], inst["stride"], flags)
        assert rc == rca and info["steps"] == inst["nsteps"]
        assert np.array_equal(q, qa) and np.array_equal(p, pa)


def test_mixed_step_counts_and_strides():
    """Zero steps, one step, and different output strides in one batch: each
    orbit gives the bits of its run alone, in the latency kernel and in the
    eight-slot kernel; a zero-step orbit has frame 0 only and no iterations.
    A step count that is not a multiple of its stride is refused."""
    d, h = 2, 2 * math.pi / 128
    ns_e = np.array([0, 1, 9, 64, 0, 13], np.int64)
    sd_e = np.array([1, 1, 3, 16, 5, 13], np.int64)
    N = BIG
    q0, p0 = _orbits(N, d, seed=31)
    ns = np.full(N, 20, np.int64)
    sd = np.full(N, 4, np.int64)
    ns[:6], sd[:6] = ns_e, sd_e

    def run(n, q, p, nsv, sdv):
        probs = [dict(kind=K.IRKGL16_KEPLER, n=1, d=d, G=1.0)] * n
        return K.Integrator(probs, record_iters=True).integrate(q, p, h, nsv, sdv)

    big = run(N, q0, p0, ns, sd)          # eight-slot kernel
    few = run(6, q0[:6 * d], p0[:6 * d], ns_e, sd_e)  # latency kernel
    assert big[3] == 0 and few[3] == 0
    off = np.concatenate([[0], np.cumsum(d * (ns_e // sd_e + 1))])
    soff = np.concatenate([[0], np.cumsum(ns_e)])
    for i in range(6):
        one = run(1, q0[i * d:(i + 1) * d], p0[i * d:(i + 1) * d], ns_e[i:i + 1], sd_e[i:i + 1])
        assert one[0].size == off[i + 1] - off[i]
        for other in (few, big):
            assert np.array_equal(one[0], other[0][off[i]:off[i + 1]])
            assert np.array_equal(one[1], other[1][off[i]:off[i + 1]])
            assert np.array_equal(one[2]["step_iters"], other[2]["step_iters"][soff[i]:soff[i + 1]])
            assert one[2]["inst_iterations"][0] == other[2]["inst_iterations"][i]
        if ns_e[i] == 0:
            assert np.array_equal(one[0], q0[i * d:(i + 1) * d])
            assert one[2]["inst_iterations"][0] == 0
    bad = K.Integrator([dict(kind=K.IRKGL16_KEPLER, n=1, d=d, G=1.0)])
    assert bad.integrate(q0[:d], p0[:d], h, 7, 3, check=False)[3] == K.IRKGL16_EINVAL

"""Serving loop (continuous batching) on the GPU: each served result is
bit-identical to the same request integrated alone, whatever else shares the
GPU, however the time slices cut it and whatever the memory cap."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import serve
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def prob(inst):
    return serve._problem(inst)


def stream(n_req, rate, seed, steps=(200, 1500), stride=100):
    reqs = W.poisson_requests(rate, n_req, seed=seed, steps_range=steps, stride=stride,
                              plummer_sizes=(64, 128))
    return reqs


def alone(inst, flags=0):
    q, p, st, rc = K.Integrator([prob(inst)], flags=flags).integrate(
        inst["q"], inst["p"], inst["h"], inst["nsteps"], inst["stride"])
    return q, p, rc


def test_served_equals_alone():
    reqs = stream(24, rate=2000.0, seed=1)
    out = serve.run_stream(reqs, cap_bytes=1 << 28, slice_steps=150, keep_frames=True)
    for (t, inst), (q, p, info, rc) in zip(reqs, out["results"]):
        qa, pa, rca = alone(inst)
        assert rc == rca
        assert info["steps"] == inst["nsteps"]
        assert np.array_equal(q, qa) and np.array_equal(p, pa), inst["cls"]
    assert out["p99_s"] >= out["p50_s"] > 0


def test_small_memory_cap_queues_and_matches():
    reqs = stream(12, rate=5000.0, seed=2)
    # room for only a few resident requests at a time
    biggest = max(inst["n"] * inst["d"] * 12 * 8 + 8 * (2 * inst["n"] + 1) for _, inst in reqs)
    out = serve.run_stream(reqs, cap_bytes=3 * biggest + 4096, slice_steps=400, keep_frames=True)
    for (t, inst), (q, p, info, rc) in zip(reqs, out["results"]):
        qa, pa, _ = alone(inst)
        assert np.array_equal(q, qa) and np.array_equal(p, pa)
    admits = sorted(r[2]["admit_s"] for r in out["results"])
    assert admits[-1] > admits[0]  # later requests waited for memory


def test_served_reproducible_matches_oracle(orc):
    reqs = stream(6, rate=1000.0, seed=3, steps=(100, 400))
    out = serve.run_stream(reqs, cap_bytes=1 << 27, slice_steps=70, keep_frames=True,
                           flags=K.IRKGL16_REPRODUCIBLE)
    for (t, inst), (q, p, info, rc) in zip(reqs, out["results"]):
        sp = orc.Spec(inst["kind"], inst["n"], inst["d"], mass=inst.get("mass"),
                      G=inst.get("G", 1.0), eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
        r = orc.integrate(sp, inst["q"], inst["p"], inst["h"], inst["nsteps"], inst["stride"])
        assert np.array_equal(q, r["q"].ravel()) and np.array_equal(p, r["p"].ravel()), inst["cls"]


def test_served_nonfinite_isolated():
    reqs = stream(6, rate=1000.0, seed=4, steps=(200, 400))
    m = np.array([1.0, 1.0])
    bad = dict(kind=K.IRKGL16_GRAVITY, n=2, d=3, mass=m, G=1.0, eps=0.0, q=np.zeros(6),
               p=np.zeros(6), h=0.1, nsteps=300, stride=100, cls="bad")
    reqs.insert(2, (reqs[1][0], bad))
    out = serve.run_stream(reqs, cap_bytes=1 << 27, slice_steps=50, keep_frames=True)
    for (t, inst), (q, p, info, rc) in zip(reqs, out["results"]):
        if inst["cls"] == "bad":
            assert rc == K.IRKGL16_ENONFINITE and np.all(np.isnan(q[6:]))
        else:
            qa, pa, _ = alone(inst)
            assert np.array_equal(q, qa) and np.array_equal(p, pa)


def test_served_whole_gpu_request_in_slices():
    inst = W.plummer(600, seed=21)
    inst.update(nsteps=6, stride=2)
    reqs = [(0.0, inst)] + stream(4, rate=1000.0, seed=5, steps=(100, 300))
    out = serve.run_stream(reqs, cap_bytes=1 << 28, slice_steps=3, keep_frames=True)
    for (t, r_inst), (q, p, info, rc) in zip(reqs, out["results"]):
        qa, pa, _ = alone(r_inst)
        assert np.array_equal(q, qa) and np.array_equal(p, pa)


def test_cancel_resident_and_pending():
    """A resident request cancelled mid-run keeps the frames of the steps it
    completed (equal to the same request alone) and NaN after them; a request
    still waiting for memory is dropped with only its initial frame; the other
    requests are untouched.  The server's slice totals are consistent."""
    import time
    long_inst = W.uneven_mix(1, seed=31, classes=[("gravity", 16)])[0]
    long_inst.update(nsteps=200000, stride=100)
    short = W.uneven_mix(1, seed=32, classes=[("gravity", 6)])[0]
    short.update(nsteps=300, stride=100)
    waiting = W.uneven_mix(1, seed=33, classes=[("gravity", 6)])[0]
    waiting.update(nsteps=300, stride=100)
    need = lambda i: 8 * (i["n"] * i["d"] * 12 + i["n"])
    # room for the long and the short request, not for the third one as well
    srv = K.Server(cap_bytes=need(long_inst) + need(short) + 1024, slice_steps=50)
    try:
        t_long = srv.submit(prob(long_inst), long_inst["q"], long_inst["p"], long_inst["h"],
                            long_inst["nsteps"], long_inst["stride"])
        t_short = srv.submit(prob(short), short["q"], short["p"], short["h"], short["nsteps"],
                             short["stride"])
        t_wait = srv.submit(prob(waiting), waiting["q"], waiting["p"], waiting["h"],
                            waiting["nsteps"], waiting["stride"])
        qs, ps, info_s, rc_s = srv.wait(t_short)
        time.sleep(0.05)
        srv.cancel(t_wait)     # may still be pending, or admitted by now
        srv.cancel(t_long)     # resident
        ql, pl, info_l, rc_l = srv.wait(t_long)
        qw, pw, info_w, rc_w = srv.wait(t_wait)
        st = srv.stats()
    finally:
        srv.close()
    qa, pa, _ = alone(short)
    assert rc_s == 0 and np.array_equal(qs, qa) and np.array_equal(ps, pa)
    assert rc_l == K.IRKGL16_ECANCELED and 0 < info_l["steps"] < long_inst["nsteps"]
    dq = long_inst["n"] * long_inst["d"]
    nf = info_l["steps"] // long_inst["stride"] + 1     # frames completed
    qla, pla, _ = alone(dict(long_inst, nsteps=(nf - 1) * long_inst["stride"]))
    assert np.array_equal(ql[:nf * dq], qla) and np.array_equal(pl[:nf * dq], pla)
    assert np.all(np.isnan(ql[nf * dq:])) and np.all(np.isnan(pl[nf * dq:]))
    assert rc_w in (0, K.IRKGL16_ECANCELED)
    if rc_w == K.IRKGL16_ECANCELED:
        dw = waiting["n"] * waiting["d"]
        nfw = info_w["steps"] // waiting["stride"] + 1
        assert np.array_equal(qw[:dw], waiting["q"]) and np.all(np.isnan(qw[nfw * dw:]))
    assert st["requests_done"] == 3 and st["requests_cancelled"] >= 1
    assert st["slices"] >= 1 and 0 < st["slice_device_s"] <= st["slice_wall_s"]

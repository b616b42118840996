"""The plain form with its step loop captured in a HIP graph (IRKGL16_PLAIN |
IRKGL16_GRAPH): every replay advances every unfinished instance by one step.
Every frame (output every step) is compared with the eager plain form and with
the batched form, on a mix of all kernel classes including a whole-GPU system
whose cooperative launches run eagerly between the replays."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def prob(inst):
    p = dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
             eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
    if inst.get("mass") is not None:
        p["mass"] = inst["mass"]
    return p


def mix():
    out = [W.kepler_c1()]
    out += W.planetary_systems(2, 6, seed=31) + W.planetary_systems(1, 16, seed=32)
    out += [W.fpu_chain(32, seed=33), W.fpu_chain(256, seed=34)]
    out += [W.plummer(600, seed=35)]
    for i, m in enumerate(out):
        if "h" not in m:
            m["h"] = 0.5
    return out


@pytest.mark.parametrize("with_large", [False, True], ids=["batched-classes", "with-whole-gpu"])
def test_graph_replay_equals_eager_plain_every_step(with_large):
    insts = mix() if with_large else mix()[:-1]
    probs = [prob(m) for m in insts]
    q0 = np.concatenate([m["q"] for m in insts])
    p0 = np.concatenate([m["p"] for m in insts])
    h = np.array([m["h"] for m in insts])
    ns = np.array([4 + 3 * (i % 4) for i in range(len(insts))], np.int64)  # uneven
    eager = K.Integrator(probs, flags=K.IRKGL16_PLAIN, record_iters=True)
    graph = K.Integrator(probs, flags=K.IRKGL16_PLAIN | K.IRKGL16_GRAPH, record_iters=True)
    batched = K.Integrator(probs, record_iters=True)
    qe, pe, se, rce = eager.integrate(q0, p0, h, ns, 1)
    qg, pg, sg, rcg = graph.integrate(q0, p0, h, ns, 1)
    qb, pb, sb, rcb = batched.integrate(q0, p0, h, ns, 1)
    assert rce == rcg == rcb
    assert np.array_equal(qe, qg) and np.array_equal(pe, pg)
    assert np.array_equal(qb, qg) and np.array_equal(pb, pg)
    assert np.array_equal(se["step_iters"], sg["step_iters"])
    assert se["steps"] == sg["steps"] == int(ns.sum())
    # a second call on the same context replays a freshly captured graph
    qg2, pg2, _, _ = graph.integrate(q0, p0, h, ns, 1)
    assert np.array_equal(qg2, qe) and np.array_equal(pg2, pe)


def test_graph_replay_reproducible_matches_oracle(orc):
    insts = mix()[:4]
    probs = [prob(m) for m in insts]
    q0 = np.concatenate([m["q"] for m in insts])
    p0 = np.concatenate([m["p"] for m in insts])
    h = np.array([m["h"] for m in insts])
    n = 12
    q, p, st, rc = K.Integrator(probs, flags=K.IRKGL16_PLAIN | K.IRKGL16_GRAPH |
                                K.IRKGL16_REPRODUCIBLE).integrate(q0, p0, h, n, 3)
    specs = [orc.Spec(m["kind"], m["n"], m["d"], mass=m.get("mass"), G=m.get("G", 1.0),
                      eps=m.get("eps", 0.0), beta=m.get("beta", 0.0)) for m in insts]
    r = orc.integrate_batch(specs, q0, p0, h, n, 3)
    assert np.array_equal(q, r["q"]) and np.array_equal(p, r["p"])

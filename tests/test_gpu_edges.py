"""Degenerate step counts in a batch of every built-in kernel class (few-body,
stage-parallel, workgroup, whole-GPU, chain, Kepler): instances with zero
steps, one step, and a single frame at the end, next to ordinary ones.  Each
instance gives the bits of its run alone; a zero-step instance has frame 0
(its input) only and no iterations."""
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


def batch():
    """(instance, steps, stride) triples: per class a zero-step, a one-step
    and a short ordinary instance."""
    by_cls = {}
    for k, (kind, size) in enumerate(W.MIX_CLASSES):
        by_cls[f"{kind}{size}"] = W.uneven_mix(3, seed=70 + k, classes=[(kind, size)])
    kep = W.kepler_c1()
    by_cls["kepler"] = [kep, dict(kep, q=np.array([0.0, 0.7]), p=np.array([-1.1, 0.0])),
                        dict(kep, q=np.array([1.2, 0.1]), p=np.array([0.1, 0.8]))]
    by_cls["plummer600"] = [W.plummer(600, seed=s) for s in (1, 2, 3)]
    out = []
    for cls in sorted(by_cls):
        insts = by_cls[cls]
        for inst in insts:
            inst["cls"] = cls
        out.append((insts[0], 0, 1))
        out.append((insts[1], 1, 1))
        out.append((insts[2], 6, 6) if cls == "plummer600" else (insts[2], 12, 4))
    return out


def test_zero_and_one_step_instances_in_every_class():
    cases = batch()
    probs = [prob(c[0]) for c in cases]
    h = np.array([c[0]["h"] for c in cases])
    ns = np.array([c[1] for c in cases], np.int64)
    sd = np.array([c[2] for c in cases], np.int64)
    q0 = np.concatenate([np.ravel(c[0]["q"]) for c in cases])
    p0 = np.concatenate([np.ravel(c[0]["p"]) for c in cases])
    print(f"edge batch: {len(cases)} instances", flush=True)
    q, p, st, rc = K.Integrator(probs, record_iters=True).integrate(q0, p0, h, ns, sd)
    assert rc in (0, K.IRKGL16_ENOCONV)
    off = soff = 0
    for i, (inst, n, s) in enumerate(cases):
        dq = inst["n"] * inst["d"]
        size = dq * (n // s + 1)
        qa, pa, sa, rca = K.Integrator([probs[i]], record_iters=True).integrate(
            np.ravel(inst["q"]), np.ravel(inst["p"]), inst["h"], n, s)
        name = inst["cls"]
        assert np.array_equal(qa, q[off:off + size]), (name, n)
        assert np.array_equal(pa, p[off:off + size]), (name, n)
        assert np.array_equal(sa["step_iters"], st["step_iters"][soff:soff + n]), (name, n)
        assert sa["inst_iterations"][0] == st["inst_iterations"][i]
        if n == 0:
            assert np.array_equal(qa, np.ravel(inst["q"])), name
            assert sa["inst_iterations"][0] == 0
        off += size
        soff += n
    assert off == q.size

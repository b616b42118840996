"""GPU parity of the workgroup-tile kernel (gravity up to 512 bodies, FPU-beta
chains up to 1024 sites) against the CPU oracle, and of mixed batches."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def prob(inst):
    p = dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
             eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
    if inst.get("mass") is not None:
        p["mass"] = inst["mass"]
    return p


def spec(orc, inst):
    return orc.Spec(inst["kind"], inst["n"], inst["d"], mass=inst.get("mass"),
                    G=inst.get("G", 1.0), eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))


def cases():
    out = []
    for nb, seed in ((16, 1), (64, 2)):
        s = W.planetary_systems(1, nb, seed=seed)[0]
        s["h"] = 1.0
        out.append((f"gravity{nb}", s, 200))
    pl = W.plummer(256, seed=7)
    out.append(("plummer256", pl, 40))
    for n, seed in ((32, 3), (256, 4), (1024, 5)):
        out.append((f"chain{n}", W.fpu_chain(n, seed=seed), 500))
    return out


@pytest.mark.parametrize("name,inst,nsteps", cases(), ids=[c[0] for c in cases()])
def test_reproducible_bit_identical(orc, name, inst, nsteps):
    integ = K.Integrator([prob(inst)], record_iters=True, flags=K.IRKGL16_REPRODUCIBLE)
    stride = max(1, nsteps // 10)
    q, p, st, rc = integ.integrate(inst["q"], inst["p"], inst["h"], nsteps, stride)
    r = orc.integrate(spec(orc, inst), inst["q"], inst["p"], inst["h"], nsteps, stride,
                      want_iters=True)
    assert rc == r["rc"]
    assert np.array_equal(q, r["q"].ravel()), name
    assert np.array_equal(p, r["p"].ravel()), name
    assert np.array_equal(st["step_iters"].astype(np.int32), r["iters"])


@pytest.mark.parametrize("name,inst,nsteps", cases(), ids=[c[0] for c in cases()])
def test_fast_within_tolerance(orc, name, inst, nsteps):
    integ = K.Integrator([prob(inst)], record_iters=True)
    q, p, st, rc = integ.integrate(inst["q"], inst["p"], inst["h"], nsteps, nsteps)
    r = orc.integrate(spec(orc, inst), inst["q"], inst["p"], inst["h"], nsteps, nsteps,
                      want_iters=True)
    q, p = q.reshape(2, -1), p.reshape(2, -1)
    # rounding sensitivity of the problem itself: the oracle's divergence under
    # 1-ulp perturbations of every initial coordinate (chaos amplifies it)
    rng = np.random.default_rng(1)
    sens_q = sens_p = 0.0
    dks = []
    for _ in range(2):
        q0 = inst["q"] + rng.choice([-1.0, 1.0], inst["q"].size) * np.spacing(np.abs(inst["q"]))
        p0 = inst["p"] + rng.choice([-1.0, 1.0], inst["p"].size) * np.spacing(np.abs(inst["p"]))
        rp = orc.integrate(spec(orc, inst), q0, p0, inst["h"], nsteps, nsteps, want_iters=True)
        sens_q = max(sens_q, relmax(rp["q"][1], r["q"][1]))
        sens_p = max(sens_p, relmax(rp["p"][1], r["p"][1]))
        dks.append(np.abs(rp["iters"].astype(int) - r["iters"]))
    assert relmax(q[1], r["q"][1]) <= max(1e-12, 30 * sens_q), (name, sens_q)
    assert relmax(p[1], r["p"][1]) <= max(1e-12, 30 * sens_p), (name, sens_p)
    # Iteration counts: within +-1 on at least 99% of the steps, unless the
    # oracle's own counts move further under the 1-ulp perturbations (the
    # stopping rule compares increments at rounding level); then no worse than
    # that.
    dk = np.abs(st["step_iters"].astype(int) - r["iters"])
    cut = 20 if max(sens_q, sens_p) > 1e-13 else len(dk)  # chaotic: before separation
    dk = dk[:cut]
    own_frac = min(float(np.mean(d[:cut] <= 1)) for d in dks)
    own_max = max(int(d[:cut].max()) for d in dks)
    assert np.mean(dk <= 1) >= min(0.99, own_frac), (name, own_frac)
    assert dk.max() <= max(3, own_max), (name, own_max)


def test_mixed_batch_equals_alone(orc):
    """Every class in one call (small-system kernel, workgroup kernel at several
    slot widths); each instance is bit-identical to a run of it alone."""
    mix = W.uneven_mix(48, seed=99)
    probs = [prob(m) for m in mix]
    h = np.array([m["h"] for m in mix])
    ns = np.full(len(mix), 60, np.int64)
    q0 = np.concatenate([m["q"] for m in mix])
    p0 = np.concatenate([m["p"] for m in mix])
    q, p, st, rc = K.Integrator(probs).integrate(q0, p0, h, ns, 20)
    off = 0
    for i, m in enumerate(mix):
        dq = m["n"] * m["d"]
        size = dq * 4
        if i % 6 == 0:
            qa, pa, _, _ = K.Integrator([probs[i]]).integrate(m["q"], m["p"], m["h"], 60, 20)
            assert np.array_equal(qa, q[off:off + size]), m["cls"]
            assert np.array_equal(pa, p[off:off + size]), m["cls"]
        off += size
    assert st["steps"] == 60 * len(mix)


def test_mixed_batch_reproducible_matches_oracle(orc):
    mix = W.uneven_mix(21, seed=5)
    probs = [prob(m) for m in mix]
    h = np.array([m["h"] for m in mix])
    n = 30
    q0 = np.concatenate([m["q"] for m in mix])
    p0 = np.concatenate([m["p"] for m in mix])
    q, p, st, rc = K.Integrator(probs, flags=K.IRKGL16_REPRODUCIBLE).integrate(q0, p0, h, n, n)
    r = orc.integrate_batch([spec(orc, m) for m in mix], q0, p0, h, n, n)
    assert np.array_equal(q, r["q"]) and np.array_equal(p, r["p"])
    assert np.array_equal(st["inst_iterations"], r["iters"])

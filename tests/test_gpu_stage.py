"""GPU parity of the stage-parallel kernel (gravitational systems of 9..128
bodies in d = 1, 2, 3; one lane per body and stage) against the CPU oracle."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def prob(inst):
    return dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
                eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0), mass=inst["mass"])


def spec(orc, inst):
    return orc.Spec(inst["kind"], inst["n"], inst["d"], mass=inst["mass"],
                    G=inst.get("G", 1.0), eps=inst.get("eps", 0.0))


def project(inst, d):
    """The same system restricted to its first d coordinates."""
    n = inst["n"]
    out = dict(inst)
    out["d"] = d
    out["q"] = np.ascontiguousarray(inst["q"].reshape(n, 3)[:, :d]).ravel()
    out["p"] = np.ascontiguousarray(inst["p"].reshape(n, 3)[:, :d]).ravel()
    return out


def cases():
    out = []
    for nb, seed in ((9, 1), (16, 2), (64, 3)):
        s = W.planetary_systems(1, nb, seed=seed)[0]
        s["h"] = 1.0
        out.append((f"planetary{nb}", s, 150))
    for n, seed in ((100, 4), (128, 5)):  # np = 104 and 128: the 1024-lane block
        pl = W.plummer(n, seed=seed)
        out.append((f"plummer{n}", pl, 40))
    s2 = project(W.planetary_systems(1, 12, seed=6)[0], 2)
    s2["h"] = 1.0
    out.append(("planar12", s2, 150))
    s5 = project(W.planetary_systems(1, 5, seed=7)[0], 2)
    s5["h"] = 1.0
    out.append(("planar5", s5, 150))
    out.append(("line24", project(W.plummer(24, seed=8), 1), 60))
    return out


CASES = cases()
IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("name,inst,nsteps", CASES, ids=IDS)
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


@pytest.mark.parametrize("name,inst,nsteps", CASES, ids=IDS)
def test_fast_within_tolerance(orc, name, inst, nsteps):
    integ = K.Integrator([prob(inst)], record_iters=True)
    q, p, st, rc = integ.integrate(inst["q"], inst["p"], inst["h"], nsteps, nsteps)
    r = orc.integrate(spec(orc, inst), inst["q"], inst["p"], inst["h"], nsteps, nsteps,
                      want_iters=True)
    q, p = q.reshape(2, -1), p.reshape(2, -1)
    # rounding sensitivity of the problem: the oracle's divergence under 1-ulp
    # perturbations of every initial coordinate
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


def test_many_instances_queue_and_plain(orc):
    """More systems than the grid holds at once (work queue), every result
    bit-identical to the reproducible oracle; the plain one-launch-per-step form
    gives the same bits."""
    systems = W.planetary_systems(40, 16, seed=11) + W.planetary_systems(30, 40, seed=12)
    for s in systems:
        s["h"] = 0.5
    probs = [prob(s) for s in systems]
    q0 = np.concatenate([s["q"] for s in systems])
    p0 = np.concatenate([s["p"] for s in systems])
    h = np.array([s["h"] for s in systems])
    ns = np.array([20 + 5 * (i % 7) for i in range(len(systems))], np.int64)
    q, p, st, rc = K.Integrator(probs, flags=K.IRKGL16_REPRODUCIBLE).integrate(q0, p0, h, ns, ns)
    r = orc.integrate_batch([spec(orc, s) for s in systems], q0, p0, h, ns, ns)
    assert np.array_equal(q, r["q"]) and np.array_equal(p, r["p"])
    sub = list(range(0, len(systems), 9))
    pq = np.concatenate([systems[i]["q"] for i in sub])
    pp = np.concatenate([systems[i]["p"] for i in sub])
    qa, pa, _, _ = K.Integrator([probs[i] for i in sub]).integrate(pq, pp, h[sub], ns[sub], ns[sub])
    qb, pb, _, _ = K.Integrator([probs[i] for i in sub], flags=K.IRKGL16_PLAIN).integrate(
        pq, pp, h[sub], ns[sub], ns[sub])
    assert np.array_equal(qa, qb) and np.array_equal(pa, pb)


def test_iteration_cap_matches_oracle(orc):
    s = W.planetary_systems(1, 16, seed=13)[0]
    s["h"] = 1.0
    integ = K.Integrator([prob(s)], max_iter=2, record_iters=True, flags=K.IRKGL16_REPRODUCIBLE)
    q, p, st, rc = integ.integrate(s["q"], s["p"], 1.0, 30, 10)
    r = orc.integrate(spec(orc, s), s["q"], s["p"], 1.0, 30, 10, max_iter=2, want_iters=True)
    assert rc == r["rc"] == K.IRKGL16_ENOCONV
    assert np.array_equal(q, r["q"].ravel()) and np.array_equal(p, r["p"].ravel())
    # steps whose increment is exactly zero at k = 2 stop there; the rest hit the cap
    assert st["nonconverged_steps"] == r["stats"]["nonconverged"] >= 1


@pytest.mark.parametrize("nb", [16, 40])  # one lane, two lanes per (body, stage)
def test_nonfinite_flagged_others_intact(nb):
    """Two coincident bodies with equal velocities: the unsoftened force is
    non-finite at the first step; that system reports ENONFINITE with NaN frames
    while a healthy system in the same call is unaffected."""
    bad = W.planetary_systems(1, nb, seed=14)[0]
    q = bad["q"].reshape(nb, 3).copy()
    v = bad["p"].reshape(nb, 3) / bad["mass"][:, None]
    q[5] = q[4]
    v[5] = v[4]
    bad["q"] = q.ravel()
    bad["p"] = (v * bad["mass"][:, None]).ravel()
    good = W.planetary_systems(1, nb, seed=15)[0]
    probs = [prob(bad), prob(good)]
    qq = np.concatenate([bad["q"], good["q"]])
    pp = np.concatenate([bad["p"], good["p"]])
    integ = K.Integrator(probs)
    q, p, st, rc = integ.integrate(qq, pp, np.array([1.0, 1.0]), 20, 10)
    assert rc == K.IRKGL16_ENONFINITE
    assert st["inst_status"][0] == K.IRKGL16_ENONFINITE and st["inst_status"][1] == 0
    dq = 3 * nb
    assert np.array_equal(q[:dq], bad["q"])      # frame 0 is the input
    assert np.all(np.isnan(q[dq:3 * dq]))         # later frames NaN
    qg, pg, _, _ = K.Integrator([probs[1]]).integrate(good["q"], good["p"], 1.0, 20, 10)
    assert np.array_equal(q[3 * dq:], qg) and np.array_equal(p[3 * dq:], pg)

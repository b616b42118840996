"""Full-size parity of the ensemble workload: 65,536 seeded six-body planetary
systems, h = 1, 10^4 steps, in one integration call as the benchmark makes it
(small-system kernel in chunks, slow instances promoted to the stage-parallel
kernel, queue ordering between chunks).  The oracle cannot run all of them in
seconds, so sampled instances -- seeded picks plus the instances that needed
the most fixed-point iterations, which are the ones promoted or evicted -- are
integrated by the oracle one by one; properties that hold at any size are
checked on every instance."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu

N_INST, NB, D, NSTEPS, H, STRIDE = 65536, 6, 3, 10_000, 1.0, 1000
DQ = NB * D
NF = NSTEPS // STRIDE + 1
REL = 1e-12


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def r12_tolerance(sens):
    """1e-12 where the oracle's own 1-ulp divergence stays below 1e-13
    (non-chaotic over these steps), else 30 times that divergence."""
    return REL if sens < 1e-13 else 30.0 * sens


@pytest.fixture(scope="module")
def full_run():
    sy = W.planetary_systems(N_INST, NB)
    q0 = np.concatenate([s["q"] for s in sy])
    p0 = np.concatenate([s["p"] for s in sy])
    probs = [dict(kind=K.IRKGL16_GRAVITY, n=NB, d=D, mass=s["mass"], G=1.0, eps=0.0) for s in sy]
    print(f"full-size ensemble: {N_INST} x {NSTEPS} steps, stride {STRIDE}", flush=True)
    q, p, st, rc = K.Integrator(probs).integrate(q0, p0, H, NSTEPS, STRIDE)
    return sy, q0, p0, q.reshape(N_INST, NF, DQ), p.reshape(N_INST, NF, DQ), st, rc


def test_every_instance_completes(full_run):
    sy, q0, p0, Q, P, st, rc = full_run
    assert rc in (0, K.IRKGL16_ENOCONV)
    assert st["steps"] == N_INST * NSTEPS
    # a step that reaches the iteration cap is reported per instance, not an error
    assert st["n_nonfinite"] == 0
    assert np.all((st["inst_status"] == 0) | (st["inst_status"] == K.IRKGL16_ENOCONV))
    assert np.all(np.isfinite(Q)) and np.all(np.isfinite(P))
    # frame 0 is the initial state
    assert np.array_equal(Q[:, 0].ravel(), q0) and np.array_equal(P[:, 0].ravel(), p0)
    k = st["inst_iterations"] / NSTEPS
    assert st["iterations"] == int(st["inst_iterations"].sum())
    assert k.min() >= 1.0 and k.max() <= 100.0


def test_linear_momentum_is_conserved_by_every_instance(full_run):
    """Gauss collocation preserves linear invariants, and the pairwise gravity
    force sums to zero, so total momentum stays at its initial value up to
    rounding (summed over 10^4 steps with compensated updates)."""
    sy, q0, p0, Q, P, st, rc = full_run
    Pb = P.reshape(N_INST, NF, NB, D)
    tot = Pb.sum(axis=2)                                  # (inst, frame, d)
    scale = np.abs(Pb).max(axis=(1, 2, 3))
    drift = np.abs(tot - tot[:, :1]).max(axis=(1, 2)) / scale
    assert drift.max() <= 1e-12, (int(drift.argmax()), float(drift.max()))


def test_sampled_instances_match_the_oracle(full_run, orc):
    sy, q0, p0, Q, P, st, rc = full_run
    rng = np.random.default_rng(20251203)
    heavy = np.argsort(st["inst_iterations"])[-4:]       # promoted / evicted ones
    pick = np.unique(np.concatenate([rng.choice(N_INST, 12, replace=False), heavy]))
    specs = [orc.Spec(orc.GRAVITY, NB, D, mass=sy[i]["mass"]) for i in pick]
    qs = np.concatenate([q0[i * DQ:(i + 1) * DQ] for i in pick])
    ps = np.concatenate([p0[i * DQ:(i + 1) * DQ] for i in pick])
    r = orc.integrate_batch(specs, qs, ps, H, NSTEPS, STRIDE)
    assert r["rc"] >= 0          # 0, or 1 when a step reached the iteration cap
    Qo, Po = r["q"].reshape(len(pick), NF, DQ), r["p"].reshape(len(pick), NF, DQ)
    # sensitivity of each sampled instance after 10^3 steps: the oracle's own
    # divergence under 1-ulp perturbations of the initial state, for q and p
    # separately
    base = orc.integrate_batch(specs, qs, ps, H, STRIDE, STRIDE)
    sens_q = np.zeros(len(pick))
    sens_p = np.zeros(len(pick))
    bq, bp = base["q"].reshape(len(pick), 2, DQ), base["p"].reshape(len(pick), 2, DQ)
    for _ in range(2):
        qp = qs + rng.choice([-1.0, 1.0], qs.size) * np.spacing(np.abs(qs))
        pp = ps + rng.choice([-1.0, 1.0], ps.size) * np.spacing(np.abs(ps))
        x = orc.integrate_batch(specs, qp, pp, H, STRIDE, STRIDE)
        xq, xp = x["q"].reshape(len(pick), 2, DQ), x["p"].reshape(len(pick), 2, DQ)
        sens_q = np.maximum(sens_q, [relmax(xq[j, 1], bq[j, 1]) for j in range(len(pick))])
        sens_p = np.maximum(sens_p, [relmax(xp[j, 1], bp[j, 1]) for j in range(len(pick))])
    # The final energy errors after 10^4 steps: the oracle's own values from
    # 1-ulp perturbations of the initial state (3 for every sampled instance,
    # 8 for those whose final state diverges under them: through a close
    # encounter at h = 1 the energy error depends on the exact path and spans
    # orders of magnitude, e.g. 8e-7 .. 9e-2 for ensemble instance 2924).
    def final_errors(js, reps):
        out = {j: [] for j in js}
        fq = {j: [] for j in js}
        cs = [specs[j] for j in js]
        cq = np.concatenate([qs[j * DQ:(j + 1) * DQ] for j in js])
        cp = np.concatenate([ps[j * DQ:(j + 1) * DQ] for j in js])
        for _ in range(reps):
            qp = cq + rng.choice([-1.0, 1.0], cq.size) * np.spacing(np.abs(cq))
            pp = cp + rng.choice([-1.0, 1.0], cp.size) * np.spacing(np.abs(cp))
            x = orc.integrate_batch(cs, qp, pp, H, NSTEPS, NSTEPS)
            xq, xp = x["q"].reshape(len(js), 2, DQ), x["p"].reshape(len(js), 2, DQ)
            for m, j in enumerate(js):
                H0 = orc.energy(specs[j], qp[m * DQ:(m + 1) * DQ], pp[m * DQ:(m + 1) * DQ])
                out[j].append(abs(orc.energy(specs[j], xq[m, 1], xp[m, 1]) / H0 - 1))
                fq[j].append(max(relmax(xq[m, 1], Qo[j, -1]), relmax(xp[m, 1], Po[j, -1])))
        return out, fq

    e_spread, div_full = final_errors(list(range(len(pick))), 3)
    chaotic = [j for j in range(len(pick)) if max(div_full[j]) > 1e-13]
    if chaotic:
        more, _ = final_errors(chaotic, 5)
        for j in chaotic:
            e_spread[j] += more[j]
    smooth = 0
    for j, i in enumerate(pick):
        H0g = orc.energy(specs[j], Q[i, 0], P[i, 0])
        eg = abs(orc.energy(specs[j], Q[i, -1], P[i, -1]) / H0g - 1)
        eo = abs(orc.energy(specs[j], Qo[j, -1], Po[j, -1]) / H0g - 1)
        kg, ko = st["inst_iterations"][i], r["iters"][j]
        if max(sens_q[j], sens_p[j]) <= 1e-13:   # non-chaotic over 10^3 steps
            smooth += 1
            assert relmax(Q[i, 1], Qo[j, 1]) <= r12_tolerance(sens_q[j]), (int(i), sens_q[j])
            assert relmax(P[i, 1], Po[j, 1]) <= r12_tolerance(sens_p[j]), (int(i), sens_p[j])
        worst = max([eo] + e_spread[j])
        if j not in chaotic:   # non-chaotic over the whole run
            assert eg <= max(1e-12, 2.0 * worst), (int(i), eg, eo, e_spread[j])
            assert abs(kg - ko) <= 0.05 * ko, (int(i), int(kg), int(ko))
        else:
            # rounding differences are amplified: the two trajectories differ
            # but are equally valid; the energy error stays within the range
            # the oracle itself reaches over 1-ulp perturbations
            assert eg <= 100.0 * max(worst, 1e-12), (int(i), eg, eo, e_spread[j])
    assert smooth >= len(pick) // 4, smooth


# ---- the uneven batch at its benchmark size: 4,096 instances of seven classes
# (gravity 3/6/16/64 bodies, FPU-beta chains 32/256/1024 sites), per-instance
# h and 1e3..1e5 steps (multiples of 100), in one call (final frames only, as
# the benchmark), except that three instances of every class -- the shortest,
# the median and the longest integration -- also write a frame at step 1000,
# where the oracle takes them up.

COMPARE_AT = 1000


def _mix_prob(m):
    p = dict(kind=m["kind"], n=m["n"], d=m["d"], G=m.get("G", 1.0), eps=m.get("eps", 0.0),
             beta=m.get("beta", 0.0))
    if m.get("mass") is not None:
        p["mass"] = m["mass"]
    return p


def _mix_spec(orc, m):
    return orc.Spec(m["kind"], m["n"], m["d"], mass=m.get("mass"), G=m.get("G", 1.0),
                    eps=m.get("eps", 0.0), beta=m.get("beta", 0.0))


def _mix_picks(mix, ns):
    pick = []
    for cls in sorted({m["cls"] for m in mix}):
        idx = sorted((i for i, m in enumerate(mix) if m["cls"] == cls), key=lambda i: (ns[i], i))
        pick += [idx[0], idx[len(idx) // 2], idx[-1]]
    return pick


@pytest.fixture(scope="module")
def mix_run():
    mix = W.uneven_mix(4096)
    h = np.array([m["h"] for m in mix])
    ns = np.array([m["nsteps"] for m in mix], np.int64)
    pick = _mix_picks(mix, ns)
    sd = ns.copy()
    sd[pick] = np.gcd(ns[pick], COMPARE_AT)     # a frame lands on step 1000
    assert np.all(ns % sd == 0) and np.all(COMPARE_AT % sd[pick] == 0)
    q0 = np.concatenate([m["q"] for m in mix])
    p0 = np.concatenate([m["p"] for m in mix])
    print(f"full-size uneven mix: {len(mix)} instances, {int(ns.sum())} steps", flush=True)
    q, p, st, rc = K.Integrator([_mix_prob(m) for m in mix]).integrate(q0, p0, h, ns, sd)
    nf = ns // sd + 1
    off = np.concatenate([[0], np.cumsum([nf[i] * m["n"] * m["d"] for i, m in enumerate(mix)])])
    return mix, h, ns, sd, pick, q0, p0, q, p, off, st, rc


def _frames(x, off, i, nf, dq):
    return x[off[i]:off[i] + nf * dq].reshape(nf, dq)


def test_mix_every_instance_completes(mix_run):
    mix, h, ns, sd, pick, q0, p0, q, p, off, st, rc = mix_run
    assert rc in (0, K.IRKGL16_ENOCONV)
    assert st["steps"] == int(ns.sum()) and st["n_nonfinite"] == 0
    assert np.all((st["inst_status"] == 0) | (st["inst_status"] == K.IRKGL16_ENOCONV))
    assert np.all(np.isfinite(q)) and np.all(np.isfinite(p))
    assert np.all(st["inst_iterations"] >= ns)


def test_mix_invariants_hold_for_every_instance(mix_run, orc):
    """At any size: the gravitational systems keep their total momentum (a
    linear invariant of the collocation method; the pair forces cancel), and
    the weakly nonlinear chains keep their energy to rounding level over up to
    10^5 steps (symplectic, no drift)."""
    mix, h, ns, sd, pick, q0, p0, q, p, off, st, rc = mix_run
    worst_mom, worst_chain = 0.0, 0.0
    for i, m in enumerate(mix):
        dq = m["n"] * m["d"]
        nf = int(ns[i] // sd[i] + 1)
        Q, P = _frames(q, off, i, nf, dq), _frames(p, off, i, nf, dq)
        if m["kind"] == W.GRAVITY:
            Pb = P.reshape(nf, m["n"], 3)
            tot = Pb.sum(axis=1)
            drift = float(np.abs(tot[-1] - tot[0]).max() / np.abs(Pb).max())
            worst_mom = max(worst_mom, drift)
        else:
            sp = _mix_spec(orc, m)
            H0 = orc.energy(sp, Q[0], P[0])
            worst_chain = max(worst_chain, abs(orc.energy(sp, Q[-1], P[-1]) / H0 - 1))
    print(f"worst momentum drift {worst_mom:.3g}, worst chain energy error {worst_chain:.3g}")
    assert worst_mom <= 1e-12
    assert worst_chain <= 1e-11


def _sensitivity(orc, specs, qs, ps, h, base, rng, reps=2):
    """The oracle's own divergence after COMPARE_AT steps under 1-ulp
    perturbations of every initial coordinate, per instance, for q and p
    separately (max-norm relative)."""
    sq = np.zeros(len(specs))
    sp = np.zeros(len(specs))
    dqs = [s.Dq for s in specs]
    offs = np.concatenate([[0], np.cumsum([2 * d for d in dqs])])
    for _ in range(reps):
        qp = qs + rng.choice([-1.0, 1.0], qs.size) * np.spacing(np.abs(qs))
        pp = ps + rng.choice([-1.0, 1.0], ps.size) * np.spacing(np.abs(ps))
        x = orc.integrate_batch(specs, qp, pp, h, COMPARE_AT, COMPARE_AT)
        for j, d in enumerate(dqs):
            a, b = offs[j] + d, offs[j] + 2 * d
            sq[j] = max(sq[j], relmax(x["q"][a:b], base["q"][a:b]))
            sp[j] = max(sp[j], relmax(x["p"][a:b], base["p"][a:b]))
    return sq, sp


def test_mix_three_of_each_class_match_the_oracle_at_step_1000(mix_run, orc):
    """Shortest, median and longest integration of every class, as run in the
    full-size call, against the oracle at step 1000: positions and momenta
    separately within the tolerance of their own rounding sensitivity, the
    energy error of eq. DHglobmax within twice the oracle's, and (for the
    instances that end at step 1000) iteration totals within 5 %."""
    mix, h, ns, sd, pick, q0, p0, q, p, off, st, rc = mix_run
    specs = [_mix_spec(orc, mix[i]) for i in pick]
    qs = np.concatenate([mix[i]["q"] for i in pick])
    ps = np.concatenate([mix[i]["p"] for i in pick])
    r = orc.integrate_batch(specs, qs, ps, h[pick], COMPARE_AT, COMPARE_AT)
    assert r["rc"] >= 0
    sens_q, sens_p = _sensitivity(orc, specs, qs, ps, h[pick], r, np.random.default_rng(20251204))
    o = 0
    compared = 0
    rows = []
    for j, i in enumerate(pick):
        m = mix[i]
        dq = m["n"] * m["d"]
        f = COMPARE_AT // int(sd[i])
        nf = int(ns[i] // sd[i] + 1)
        qg, pg = _frames(q, off, i, nf, dq), _frames(p, off, i, nf, dq)
        qo, po = r["q"][o:o + 2 * dq].reshape(2, dq), r["p"][o:o + 2 * dq].reshape(2, dq)
        o += 2 * dq
        assert np.array_equal(qg[0], qo[0]) and np.array_equal(pg[0], po[0])
        dev_q, dev_p = relmax(qg[f], qo[1]), relmax(pg[f], po[1])
        rows.append((m["cls"], int(ns[i]), dev_q, sens_q[j], dev_p, sens_p[j]))
        H0 = orc.energy(specs[j], qg[0], pg[0])
        eg = abs(orc.energy(specs[j], qg[f], pg[f]) / H0 - 1)
        eo = abs(orc.energy(specs[j], qo[1], po[1]) / H0 - 1)
        if max(sens_q[j], sens_p[j]) < 1e-10:
            compared += 1
            assert dev_q <= r12_tolerance(sens_q[j]), rows[-1]
            assert dev_p <= r12_tolerance(sens_p[j]), rows[-1]
            assert eg <= max(1e-12, 2.0 * eo), (m["cls"], eg, eo)
            if ns[i] == COMPARE_AT:
                kg, ko = st["inst_iterations"][i], r["iters"][j]
                assert abs(kg - ko) <= 0.05 * ko, (m["cls"], int(kg), int(ko))
        elif eo <= 1e-6:
            # chaotic: rounding differences are amplified; the trajectories
            # differ but are equally valid, so the energy error stays of the
            # same order
            assert eg <= 100.0 * max(eo, 1e-12), (m["cls"], eg, eo)
        # else: an encounter the step size does not resolve dominates both
        # runs' energy errors (truncation, not rounding); only finiteness holds
    for row in rows:
        print("%-10s steps %6d  dq %.2e (sens %.2e)  dp %.2e (sens %.2e)" % row)
    # every chain and the three-body systems stay far from chaos over 10^3
    # steps of this workload (the oracle's own 1-ulp divergence < 1e-11)
    assert compared >= 12, compared

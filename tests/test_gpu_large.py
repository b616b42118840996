"""GPU parity of the whole-GPU path for one large gravitational system
(N > 512 bodies; the N = 2048 Plummer cluster of the single-large-system
workload) against the CPU oracle."""
import hashlib
import os

import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def run(inst, nsteps, stride, flags=0, record=True):
    prob = dict(kind=K.IRKGL16_GRAVITY, n=inst["n"], d=3, mass=inst["mass"], G=inst["G"],
                eps=inst["eps"])
    return K.Integrator([prob], record_iters=record, flags=flags).integrate(
        inst["q"], inst["p"], inst["h"], nsteps, stride)


def oracle_spec(orc, inst):
    return orc.Spec(orc.GRAVITY, inst["n"], 3, mass=inst["mass"], G=inst["G"], eps=inst["eps"])


def oracle_run(orc, inst, nsteps, stride, iters=True, q0=None, p0=None):
    q0 = inst["q"] if q0 is None else q0
    p0 = inst["p"] if p0 is None else p0
    return orc.integrate(oracle_spec(orc, inst), q0, p0, inst["h"], nsteps, stride,
                         want_iters=iters)


# ---- the single-large-system workload itself (Plummer N = 2048, default
# seed, eps = 1e-2, h = 1e-3): parity over 10^2 steps, energy statistics over
# 10^3 steps against figures the oracle wrote (tests/golden/make_c3_golden.py)

C3_STEPS, C3_STRIDE = 100, 10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "c3_plummer2048_1000.txt")


def read_golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or "=" not in line:
            continue
        k, v = (x.strip() for x in line.split("=", 1))
        out[k] = float.fromhex(v) if v.startswith("0x") else v
    return out


def dd_energy_errors(orc, inst, q, p):
    """|H_n - H_0| / |H_0| of every frame, H in double-double arithmetic from
    the binary64 frame (eq. DHglobmax)."""
    sp = oracle_spec(orc, inst)
    z = np.zeros(q.shape[1])
    H = [orc.energy_dd(sp, q[f], z, p[f], z) for f in range(q.shape[0])]
    H0 = H[0][0] + H[0][1]
    return np.array([abs((h[0] - H[0][0]) + (h[1] - H[0][1])) / abs(H0) for h in H])


@pytest.fixture(scope="module")
def c3_oracle(orc):
    inst = W.plummer(2048)
    print(f"oracle: Plummer 2048, {C3_STEPS} steps", flush=True)
    r = oracle_run(orc, inst, C3_STEPS, C3_STRIDE)
    return inst, r


def test_c3_reproducible_bit_identical_over_100_steps(orc, c3_oracle):
    inst, r = c3_oracle
    q, p, st, rc = run(inst, C3_STEPS, C3_STRIDE, flags=K.IRKGL16_REPRODUCIBLE)
    assert rc == r["rc"] == 0
    assert np.array_equal(q, r["q"].ravel()) and np.array_equal(p, r["p"].ravel())
    assert np.array_equal(st["step_iters"].astype(np.int32), r["iters"])


def test_c3_fused_matches_oracle_over_100_steps(orc, c3_oracle):
    """Default arithmetic against the strict-IEEE oracle on every frame of 10^2
    steps: positions and momenta within 1e-12, or 30 times the oracle's own
    divergence under 1-ulp perturbations of the initial state where that is
    larger (the cluster is chaotic); iteration counts within +-1 per step."""
    inst, r = c3_oracle
    q, p, st, rc = run(inst, C3_STEPS, C3_STRIDE)
    assert rc == 0
    nf = C3_STEPS // C3_STRIDE + 1
    q, p = q.reshape(nf, -1), p.reshape(nf, -1)
    rng = np.random.default_rng(2048)
    sens_q = np.zeros(nf)
    sens_p = np.zeros(nf)
    for _ in range(2):
        q0 = inst["q"] + rng.choice([-1.0, 1.0], inst["q"].size) * np.spacing(np.abs(inst["q"]))
        p0 = inst["p"] + rng.choice([-1.0, 1.0], inst["p"].size) * np.spacing(np.abs(inst["p"]))
        x = oracle_run(orc, inst, C3_STEPS, C3_STRIDE, iters=False, q0=q0, p0=p0)
        sens_q = np.maximum(sens_q, [relmax(x["q"][f], r["q"][f]) for f in range(nf)])
        sens_p = np.maximum(sens_p, [relmax(x["p"][f], r["p"][f]) for f in range(nf)])
    for f in range(1, nf):
        dq, dp = relmax(q[f], r["q"][f]), relmax(p[f], r["p"][f])
        print(f"step {f * C3_STRIDE}: dq {dq:.2e} (sens {sens_q[f]:.2e}) "
              f"dp {dp:.2e} (sens {sens_p[f]:.2e})")
        assert dq <= max(1e-12, 30.0 * sens_q[f]), (f, dq, sens_q[f])
        assert dp <= max(1e-12, 30.0 * sens_p[f]), (f, dp, sens_p[f])
    dk = np.abs(st["step_iters"].astype(int) - r["iters"])
    assert dk.max() <= 1, dk.max()


def test_c3_energy_statistics_over_1000_steps(orc):
    """10^3 steps with frames every 50: the reproducible mode writes the
    oracle's frames bit for bit (SHA-256 of the frames the oracle wrote), and
    the default mode's energy errors (eq. DHglobmax: maximum and RMS over the
    frames) are at most twice the oracle's."""
    g = read_golden()
    inst = W.plummer(2048)
    n, sd = int(g["nsteps"]), int(g["stride"])
    nf = n // sd + 1
    q, p, st, rc = run(inst, n, sd, flags=K.IRKGL16_REPRODUCIBLE, record=False)
    assert rc == 0 and st["iterations"] == int(g["iterations"])
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(q, "<f8").tobytes())
    h.update(np.ascontiguousarray(p, "<f8").tobytes())
    assert h.hexdigest() == g["frames_sha256"]
    q, p, st, rc = run(inst, n, sd, record=False)
    assert rc == 0
    dH = dd_energy_errors(orc, inst, q.reshape(nf, -1), p.reshape(nf, -1))[1:]
    mx, rms = float(dH.max()), float(np.sqrt(np.mean(dH ** 2)))
    print(f"energy error: GPU max {mx:.3g} rms {rms:.3g}; "
          f"oracle max {g['dH_max']:.3g} rms {g['dH_rms']:.3g}")
    assert mx <= 2.0 * g["dH_max"] and rms <= 2.0 * g["dH_rms"]


@pytest.mark.parametrize("n,nsteps", [(600, 6), (2048, 3)])
def test_large_reproducible_bit_identical(orc, n, nsteps):
    inst = W.plummer(n, seed=11)
    q, p, st, rc = run(inst, nsteps, 1, flags=K.IRKGL16_REPRODUCIBLE)
    r = oracle_run(orc, inst, nsteps, 1)
    assert rc == 0
    assert np.array_equal(q, r["q"].ravel()) and np.array_equal(p, r["p"].ravel())
    assert np.array_equal(st["step_iters"].astype(np.int32), r["iters"])


def test_large_fast_matches_oracle(orc):
    inst = W.plummer(2048, seed=3)
    n = 4
    q, p, st, rc = run(inst, n, n)
    r = oracle_run(orc, inst, n, n)
    assert rc == 0
    q, p = q.reshape(2, -1), p.reshape(2, -1)
    assert relmax(q[1], r["q"][1]) <= 1e-14
    assert relmax(p[1], r["p"][1]) <= 1e-12
    assert np.abs(st["step_iters"].astype(int) - r["iters"]).max() <= 1


def test_large_plain_equals_batched():
    inst = W.plummer(700, seed=5)
    a = run(inst, 3, 1)
    b = run(inst, 3, 1, flags=K.IRKGL16_PLAIN)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_large_nonfinite_stops_cleanly():
    inst = W.plummer(600, seed=8)
    inst = dict(inst)
    inst["eps"] = 0.0
    q, p = inst["q"].copy(), inst["p"].copy()
    q[3:6] = q[0:3]  # bodies 0 and 1 coincide and move together (equal masses):
    p[3:6] = p[0:3]  # every stage has r = 0 between them, without softening
    inst["q"], inst["p"] = q, p
    qo, po, st, rc = run(inst, 4, 1)
    assert rc == K.IRKGL16_ENONFINITE
    assert np.all(np.isnan(qo.reshape(5, -1)[1:]))


@pytest.mark.parametrize("n", [513, 1001])
def test_large_ragged_last_group_reproducible(orc, n):
    """Body counts that leave a partial last group of 8 targets."""
    inst = W.plummer(n, seed=17)
    q, p, st, rc = run(inst, 3, 1, flags=K.IRKGL16_REPRODUCIBLE)
    r = oracle_run(orc, inst, 3, 1)
    assert rc == 0
    assert np.array_equal(q, r["q"].ravel()) and np.array_equal(p, r["p"].ravel())
    assert np.array_equal(st["step_iters"].astype(np.int32), r["iters"])


def test_large_several_groups_per_workgroup(orc):
    """4100 bodies: more target groups than co-resident workgroups, so a
    workgroup integrates several groups (one state wavefront each)."""
    inst = W.plummer(4100, seed=19)
    q, p, st, rc = run(inst, 2, 2)
    r = oracle_run(orc, inst, 2, 2)
    assert rc == 0
    q, p = q.reshape(2, -1), p.reshape(2, -1)
    assert relmax(q[1], r["q"][1]) <= 1e-14
    assert relmax(p[1], r["p"][1]) <= 1e-12
    assert np.abs(st["step_iters"].astype(int) - r["iters"]).max() <= 1


def test_large_resumed_launches_equal_one_launch():
    """Integrating 6 steps as 6 one-step launches (state, increments and
    counters resumed from device memory) gives the bits of one 6-step launch."""
    inst = W.plummer(1500, seed=23)
    a = run(inst, 6, 2)
    b = run(inst, 6, 2, flags=K.IRKGL16_PLAIN)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert a[2]["iterations"] == b[2]["iterations"]

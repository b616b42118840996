"""GPU parity of the s-stage members of the family (s = 2, 4, 6: IRKGL4,
IRKGL8, IRKGL12; irkgl16_options.stages) on the run-time compiled kernels,
against the oracle's s-stage integrators, through the C ABI.

Reproducible mode is bit-identical to the oracle for every s in both forms
and on both kernels (one instance per lane for Dq <= 4, 8-lane slots above,
where lanes past the stage count idle in the stage role); the default fused
mode meets the rounding-level bar; plain, graph and batched forms agree."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import user_forces as UF
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu

STAGES = (2, 4, 6)


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("s", STAGES)
def test_henon_heiles_bitwise(orc, s):
    n_inst, nsteps, stride = 29, 600, 60
    q0, p0 = W.henon_heiles_ensemble(n_inst, seed=60 + s, energy=(0.02, 1 / 12),
                                     q2_range=(-0.1, 0.3), p2_range=(-0.1, 0.2))
    h = 2 * np.pi / 128
    integ = K.Integrator.user(UF.HENON_HEILES, 2, n_inst, flags=K.IRKGL16_REPRODUCIBLE,
                              record_iters=True, stages=s)
    q, p, st, rc = integ.integrate(q0.ravel(), p0.ravel(), h, nsteps, stride)
    assert rc == 0
    r = orc.integrate_batch([orc.Spec(orc.HENON, 1, 2)] * n_inst, q0.ravel(), p0.ravel(), h,
                            nsteps, stride, s=s)
    assert r["rc"] == 0
    assert np.array_equal(q, r["q"]) and np.array_equal(p, r["p"])
    one = orc.integrate_s(orc.Spec(orc.HENON, 1, 2), s, q0[0], p0[0], h, nsteps, stride,
                          want_iters=True)
    assert np.array_equal(st["step_iters"][:nsteps].astype(int), one["iters"])


@pytest.mark.parametrize("s", STAGES)
def test_harmonic_slot_kernel_bitwise(orc, s):
    """Dq = 13: the 8-lane-slot kernel with two components per lane."""
    n_inst, dq, nsteps, stride = 11, 13, 200, 20
    rng = np.random.default_rng(70 + s)
    w2 = rng.uniform(0.3, 3.0, n_inst)
    q0 = rng.standard_normal(n_inst * dq)
    p0 = rng.standard_normal(n_inst * dq)
    integ = K.Integrator.user(UF.HARMONIC, dq, n_inst, params=w2[:, None],
                              flags=K.IRKGL16_REPRODUCIBLE, stages=s)
    q, p, st, rc = integ.integrate(q0, p0, 0.2, nsteps, stride)
    assert rc == 0
    specs = [orc.Spec(orc.HARMONIC, dq, 1, G=w2[i]) for i in range(n_inst)]
    r = orc.integrate_batch(specs, q0, p0, 0.2, nsteps, stride, s=s)
    assert np.array_equal(q, r["q"]) and np.array_equal(p, r["p"])


@pytest.mark.parametrize("s", STAGES)
@pytest.mark.parametrize("D", [4, 10])
def test_first_order_bitwise(orc, s, D):
    """First-order form: Kepler (D = 4, lane kernel) and a 5-dimensional
    oscillator (D = 10, slot kernel)."""
    n_inst, nsteps, stride = 13, 500, 50
    rng = np.random.default_rng(80 + s + D)
    if D == 4:
        y0 = np.concatenate([[r, 0.0, 0.0, np.sqrt(0.9 / r)] for r in rng.uniform(0.7, 1.3, n_inst)])
        src, prm = UF.KEPLER_RHS, np.ones((n_inst, 1))
        specs = [orc.Spec(orc.ODE_KEPLER, 2, 2, G=1.0)] * n_inst
        h = 2 * np.pi / 256
    else:
        y0 = rng.standard_normal(n_inst * D)
        w2 = rng.uniform(0.3, 2.0, n_inst)
        src, prm = UF.OSC_RHS, w2[:, None]
        specs = [orc.Spec(orc.ODE_OSC, 2, D // 2, G=w) for w in w2]
        h = 0.2
    integ = K.Integrator.ode(src, D, n_inst, params=prm, flags=K.IRKGL16_REPRODUCIBLE, stages=s)
    y, _, st, rc = integ.integrate(y0, None, h, nsteps, stride)
    assert rc == 0
    r = orc.integrate_ode_batch(specs, y0, h, nsteps, stride, s=s)
    assert r["rc"] == 0
    assert np.array_equal(y, r["y"])


@pytest.mark.parametrize("s", STAGES)
def test_fused_mode_within_tolerance(orc, s):
    n_inst, nsteps = 32, 1000
    q0, p0 = W.henon_heiles_ensemble(n_inst, seed=90 + s, energy=(0.02, 0.06),
                                     q2_range=(-0.1, 0.3), p2_range=(-0.1, 0.2))
    h = 2 * np.pi / 128
    integ = K.Integrator.user(UF.HENON_HEILES, 2, n_inst, stages=s)
    q, p, st, rc = integ.integrate(q0.ravel(), p0.ravel(), h, nsteps, nsteps)
    r = orc.integrate_batch([orc.Spec(orc.HENON, 1, 2)] * n_inst, q0.ravel(), p0.ravel(), h,
                            nsteps, nsteps, s=s)
    q, rq = q.reshape(n_inst, 2, 2), r["q"].reshape(n_inst, 2, 2)
    for i in range(n_inst):
        assert relmax(q[i, -1], rq[i, -1]) <= 1e-12, i


def test_stage_count_changes_the_method_and_eight_is_default():
    n_inst = 8
    q0, p0 = W.henon_heiles_ensemble(n_inst, seed=99)
    h = 0.3
    outs = {}
    for s in (0, 8, 4):
        integ = K.Integrator.user(UF.HENON_HEILES, 2, n_inst, flags=K.IRKGL16_REPRODUCIBLE,
                                  stages=s)
        outs[s] = integ.integrate(q0.ravel(), p0.ravel(), h, 200, 200)
    assert np.array_equal(outs[0][0], outs[8][0]) and np.array_equal(outs[0][1], outs[8][1])
    assert not np.array_equal(outs[4][0], outs[8][0])


@pytest.mark.parametrize("s", [2, 6])
def test_plain_graph_batched_agree(s):
    n_inst = 10
    q0, p0 = W.henon_heiles_ensemble(n_inst, seed=100 + s)
    ns = np.array([4 + 5 * (i % 3) for i in range(n_inst)], np.int64)
    outs = []
    for flags in (0, K.IRKGL16_PLAIN, K.IRKGL16_PLAIN | K.IRKGL16_GRAPH):
        integ = K.Integrator.user(UF.HENON_HEILES, 2, n_inst, flags=flags, record_iters=True,
                                  stages=s)
        outs.append(integ.integrate(q0.ravel(), p0.ravel(), 2 * np.pi / 64, ns, 1))
    for q, p, st, rc in outs[1:]:
        assert np.array_equal(q, outs[0][0]) and np.array_equal(p, outs[0][1])
        assert np.array_equal(st["step_iters"], outs[0][2]["step_iters"])

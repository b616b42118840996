"""GPU parity of the first-order (mu) form, y' = f(t, y), with right-hand
sides compiled at run time (irkgl16_create_ode), against the first-order CPU
oracle, through the C ABI.

Reproducible mode matches the oracle bit for bit when the right-hand side is
the same expression (oscillator, Kepler, damped system; D from 2 to 16, on
the one-instance-per-lane kernel for D <= 4 and the 8-lane-slot kernel
above); where the device and host trigonometric functions may differ in the
last bit (the driven system, the Schwarzschild problem) and in the default
fused mode, the bar is the rounding-level one: max relative difference
<= 1e-12 after 10^3 steps on regular orbits, iteration counts within +-1 on
>= 99.5 % of the steps.  Plain, graph-replayed and batched forms agree bit
for bit; an instance alone equals the same instance in a batch."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import user_forces as UF
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu

REL = 1e-12


def relmax(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def sbh_states(n, seed):
    """Schwarzschild states near the paper's regular orbit (section 5.1.1)."""
    return W.schwarzschild_ensemble(n, seed=seed), W.SBH_PARAMS


@pytest.mark.parametrize("d", [1, 2, 3, 4, 8])
def test_oscillator_bitwise(orc, d):
    """D = 2d from 2 (lane kernel) to 16 (slot kernel, two components per
    lane); per-instance frequencies; 21 instances (not a multiple of 8)."""
    n_inst, nsteps, stride = 21, 300, 30
    D = 2 * d
    rng = np.random.default_rng(200 + d)
    w2 = rng.uniform(0.3, 3.0, n_inst)
    y0 = rng.standard_normal(n_inst * D)
    integ = K.Integrator.ode(UF.OSC_RHS, D, n_inst, params=w2[:, None],
                             flags=K.IRKGL16_REPRODUCIBLE, record_iters=True)
    y, _, st, rc = integ.integrate(y0, None, 0.3, nsteps, stride)
    assert rc == 0
    specs = [orc.Spec(orc.ODE_OSC, 2, d, G=w2[i]) for i in range(n_inst)]
    r = orc.integrate_ode_batch(specs, y0, 0.3, nsteps, stride)
    assert r["rc"] == 0
    assert np.array_equal(y, r["y"])
    one = orc.integrate_ode(specs[3], y0[3 * D:4 * D], 0.3, nsteps, stride, want_iters=True)
    assert np.array_equal(st["step_iters"][3 * nsteps:4 * nsteps].astype(int), one["iters"])


@pytest.mark.parametrize("d", [2, 3])
def test_kepler_bitwise(orc, d):
    n_inst, nsteps, stride = 19, 1000, 100
    D = 2 * d
    rng = np.random.default_rng(300 + d)
    y0 = []
    for _ in range(n_inst):  # bound orbits: |v|^2 < 2/|q| * 0.8
        q = rng.uniform(0.5, 1.5) * np.array([1.0, 0.0, 0.0][:d])
        v = np.sqrt(0.8 / np.linalg.norm(q)) * np.array([0.0, 1.0, 0.2][:d])
        y0.append(np.concatenate([q, v]))
    y0 = np.concatenate(y0)
    h = 2 * np.pi / 128
    integ = K.Integrator.ode(UF.KEPLER_RHS, D, n_inst, params=np.ones((n_inst, 1)),
                             flags=K.IRKGL16_REPRODUCIBLE, record_iters=True)
    y, _, st, rc = integ.integrate(y0, None, h, nsteps, stride)
    assert rc == 0
    specs = [orc.Spec(orc.ODE_KEPLER, 2, d, G=1.0)] * n_inst
    r = orc.integrate_ode_batch(specs, y0, h, nsteps, stride)
    assert np.array_equal(y, r["y"])


def test_damped_and_stopping_rule_case_bitwise(orc):
    """The non-Hamiltonian damped system, and the oscillator from (1, 0),
    where the rule as written stops the first step after 4 iterations: the
    GPU takes the same decisions."""
    beta = np.array([0.0, 0.1, 0.3, 1.0, 2.5])
    y0 = np.tile([0.7, -0.2], len(beta))
    integ = K.Integrator.ode(UF.DAMPED_RHS, 2, len(beta), params=beta[:, None],
                             flags=K.IRKGL16_REPRODUCIBLE, record_iters=True)
    y, _, st, rc = integ.integrate(y0, None, 0.4, 300, 10)
    specs = [orc.Spec(orc.ODE_DAMPED, 1, 2, beta=b) for b in beta]
    r = orc.integrate_ode_batch(specs, y0, 0.4, 300, 10)
    assert np.array_equal(y, r["y"])
    osc = K.Integrator.ode(UF.OSC_RHS, 2, 1, params=np.ones((1, 1)),
                           flags=K.IRKGL16_REPRODUCIBLE, record_iters=True)
    y, _, st, rc = osc.integrate(np.array([1.0, 0.0]), None, 0.5, 12, 1)
    ro = orc.integrate_ode(orc.Spec(orc.ODE_OSC, 2, 1, G=1.0), [1.0, 0.0], 0.5, 12, 1,
                           want_iters=True)
    assert st["step_iters"][0] == 4 and np.array_equal(st["step_iters"].astype(int), ro["iters"])
    assert np.array_equal(y.reshape(-1, 2), ro["y"])


@pytest.mark.parametrize("fused", [False, True], ids=["reproducible", "fused"])
def test_schwarzschild_against_oracle(orc, fused):
    """Eq. Ham_SBH near the paper's regular orbit, 10^3 steps of h = 2."""
    n_inst, nsteps, stride = 32, 1000, 100
    Y0, (E, L, b) = sbh_states(n_inst, 7)
    prm = np.tile([E, L, b], (n_inst, 1))
    flags = 0 if fused else K.IRKGL16_REPRODUCIBLE
    integ = K.Integrator.ode(UF.SCHWARZSCHILD_RHS, 4, n_inst, params=prm, flags=flags,
                             record_iters=True)
    y, _, st, rc = integ.integrate(Y0.ravel(), None, 2.0, nsteps, stride)
    assert rc == 0
    spec = orc.Spec(orc.ODE_SBH, 1, 4, G=E, eps=L, beta=b)
    r = orc.integrate_ode_batch([spec] * n_inst, Y0.ravel(), 2.0, nsteps, stride)
    nf = nsteps // stride + 1
    y, ry = y.reshape(n_inst, nf, 4), r["y"].reshape(n_inst, nf, 4)
    for i in range(n_inst):
        assert relmax(y[i, -1], ry[i, -1]) <= REL, i
        H = [orc.energy_ode(spec, v) for v in y[i]]
        assert np.abs(np.array(H) + 0.5).max() < 5e-14, i
    k = st["step_iters"].reshape(n_inst, nsteps).astype(int)
    for i in range(0, n_inst, 5):
        ko = orc.integrate_ode(spec, Y0[i], 2.0, nsteps, stride, want_iters=True)["iters"]
        dk = np.abs(k[i] - ko)
        assert np.mean(dk <= 1) >= 0.995 and dk.max() <= 3, i


def test_driven_closed_form(orc):
    n_inst, nsteps, stride = 9, 400, 40
    G = np.linspace(-2.0, 2.0, n_inst)
    rng = np.random.default_rng(12)
    y0 = rng.standard_normal((n_inst, 2))
    for h in (0.5, -0.25):
        integ = K.Integrator.ode(UF.DRIVEN_RHS, 2, n_inst, params=G[:, None],
                                 flags=K.IRKGL16_REPRODUCIBLE)
        y, _, st, rc = integ.integrate(y0.ravel(), None, h, nsteps, stride)
        assert rc == 0
        y = y.reshape(n_inst, -1, 2)
        t = (np.arange(nsteps // stride + 1) * stride * h)[None, :]
        x = y0[:, :1] + y0[:, 1:] * t + G[:, None] * (1 - np.cos(t))
        assert np.abs(y[:, :, 0] - x).max() < 1e-11
        specs = [orc.Spec(orc.ODE_DRIVEN, 1, 2, G=g) for g in G]
        r = orc.integrate_ode_batch(specs, y0.ravel(), h, nsteps, stride)
        assert relmax(y.ravel(), r["y"]) <= REL


@pytest.mark.parametrize("D", [4, 6])
def test_plain_graph_batched_and_alone_agree(D):
    n_inst = 11
    rng = np.random.default_rng(40 + D)
    w2 = rng.uniform(0.5, 2.0, n_inst)
    y0 = rng.standard_normal(n_inst * D)
    ns = np.array([5 + 6 * (i % 4) for i in range(n_inst)], np.int64)
    outs = []
    for flags in (0, K.IRKGL16_PLAIN, K.IRKGL16_PLAIN | K.IRKGL16_GRAPH):
        integ = K.Integrator.ode(UF.OSC_RHS, D, n_inst, params=w2[:, None], flags=flags,
                                 record_iters=True)
        outs.append(integ.integrate(y0, None, 0.3, ns, 1))
    for y, _, st, rc in outs[1:]:
        assert rc == outs[0][3]
        assert np.array_equal(y, outs[0][0])
        assert np.array_equal(st["step_iters"], outs[0][2]["step_iters"])
    i = 4
    alone = K.Integrator.ode(UF.OSC_RHS, D, 1, params=w2[i:i + 1, None])
    ya, _, _, _ = alone.integrate(y0[i * D:(i + 1) * D], None, 0.3, ns[i], 1)
    off = int(sum(D * (ns[j] + 1) for j in range(i)))
    assert np.array_equal(ya, outs[0][0][off:off + ya.size])


def test_p_arguments_are_ignored():
    """A first-order context neither reads p0 nor writes p_out (C ABI called
    directly with both given)."""
    integ = K.Integrator.ode(UF.DAMPED_RHS, 2, 3, params=np.full((3, 1), 0.2))
    y0 = np.array([1.0, 0.0, 0.5, 0.5, -1.0, 0.2])
    a = integ.integrate(y0, None, 0.3, 20, 20)
    h = np.full(3, 0.3)
    ns = np.full(3, 20, np.int64)
    p_junk = np.full(6, np.nan)
    q_out = np.empty(12)
    p_out = np.full(12, 7.0)
    rc = K.irkgl16_integrate(integ.ctx, y0, p_junk, h, ns, ns, q_out, p_out)
    assert rc == 0
    assert np.array_equal(a[0], q_out)
    assert np.all(p_out == 7.0)
    rc = K.irkgl16_integrate(integ.ctx, y0, None, h, ns, ns, q_out, None)
    assert rc == 0 and np.array_equal(a[0], q_out)


def test_create_ode_rejects_bad_source_on_gpu():
    with pytest.raises(K.IRKGL16Error) as e:
        K.Integrator.ode(UF.HENON_HEILES, 2, 4)  # a second-order force, not f(t, y)
    assert e.value.code == K.IRKGL16_EINVAL

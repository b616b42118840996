"""Edge cases of the run-time compiled paths (user forces, first-order
right-hand sides, explicit baselines): an instance that goes non-finite stops
alone, with its later frames NaN and the others unaffected; empty batches and
zero-step calls; the iteration cap; device-pointer mode on a caller's stream.
Failures are forced through the inputs (the kernels always exit normally)."""
import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import user_forces as UF
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu

# q'' = -q until |q| exceeds 2, then the force is NaN (a blow-up signal)
BLOWUP = r"""
__device__ void irkgl16_user_force(const double* q, double* g, const double* prm, double t) {
  (void)t;
  for (int k = 0; k < IRKGL16_DQ; ++k)
    g[k] = fabs(q[k]) > 2.0 ? __builtin_nan("") : -prm[0] * q[k];
}
"""


@pytest.mark.parametrize("dq", [2, 9])
@pytest.mark.parametrize("method", [0, K.IRKGL16_SUZ90])
def test_nonfinite_instance_stops_alone(orc, dq, method):
    """Instance 1 starts beyond the threshold region's reach: its amplitude
    grows past 2 under an (unphysical) negative stiffness, the force turns
    NaN, the instance stops with ENONFINITE and NaN frames; the others match
    a run without it."""
    n_inst, nsteps, stride = 5, 200, 20
    w2 = np.array([1.0, -1.0, 0.5, 2.0, 1.5])[:, None]
    rng = np.random.default_rng(1)
    q0 = rng.uniform(-0.5, 0.5, n_inst * dq)
    p0 = rng.uniform(-0.5, 0.5, n_inst * dq)
    integ = K.Integrator.user(BLOWUP, dq, n_inst, params=w2, method=method,
                              flags=K.IRKGL16_REPRODUCIBLE)
    q, p, st, rc = integ.integrate(q0, p0, 0.1, nsteps, stride, check=False)
    assert rc == K.IRKGL16_ENONFINITE
    assert st["n_nonfinite"] == 1
    assert list(st["inst_status"]) == [0, K.IRKGL16_ENONFINITE, 0, 0, 0]
    nf = nsteps // stride + 1
    q = q.reshape(n_inst, nf, dq)
    assert np.isnan(q[1, -1]).all() and np.isfinite(q[1, 0]).all()
    keep = [0, 2, 3, 4]
    ref = K.Integrator.user(BLOWUP, dq, 4, params=w2[keep], method=method,
                            flags=K.IRKGL16_REPRODUCIBLE)
    qr, pr, _, rcr = ref.integrate(q0.reshape(n_inst, dq)[keep].ravel(),
                                   p0.reshape(n_inst, dq)[keep].ravel(), 0.1, nsteps, stride)
    assert rcr == 0
    assert np.array_equal(q[keep].ravel(), qr)


@pytest.mark.parametrize("maker", ["user", "ode", "split"])
def test_empty_batch_and_zero_steps(maker):
    if maker == "ode":
        mk = lambda n: K.Integrator.ode(UF.OSC_RHS, 2, n, params=np.ones((max(n, 1), 1))[:n]
                                         if n else None)
    elif maker == "split":
        mk = lambda n: K.Integrator.user(UF.HENON_HEILES, 2, n, method=K.IRKGL16_STRANG)
    else:
        mk = lambda n: K.Integrator.user(UF.HENON_HEILES, 2, n)
    empty = mk(0)
    q, p, st, rc = empty.integrate(np.zeros(0), np.zeros(0), np.zeros(0), np.zeros(0, np.int64),
                                   np.ones(0, np.int64))
    assert rc == 0 and q.size == 0 and st["steps"] == 0
    integ = mk(3)
    y0 = np.arange(6, dtype=float) * 0.1
    q, p, st, rc = integ.integrate(y0, y0 * 0.5, 0.1, 0, 1)
    assert rc == 0 and st["steps"] == 0
    assert np.array_equal(q, y0)  # frame 0 only


def test_iteration_cap_reported():
    """max_iter = 1 caps every step of the implicit method: the call reports
    ENOCONV (a warning) and counts the capped steps."""
    q0, p0 = W.henon_heiles_ensemble(8, seed=5)
    integ = K.Integrator.user(UF.HENON_HEILES, 2, 8, max_iter=1)
    q, p, st, rc = integ.integrate(q0.ravel(), p0.ravel(), 0.3, 50, 50, check=False)
    assert rc == K.IRKGL16_ENOCONV
    assert st["nonconverged_steps"] == 8 * 50 and st["max_k"] == 1


def test_device_pointer_mode_on_caller_stream():
    """IRKGL16_DEVICE_PTRS with a torch stream: same results as host mode."""
    import torch
    q0, p0 = W.henon_heiles_ensemble(40, seed=6)
    host = K.Integrator.user(UF.HENON_HEILES, 2, 40)
    qh, ph, _, _ = host.integrate(q0.ravel(), p0.ravel(), 0.2, 100, 10)
    stream = torch.cuda.Stream()
    dev = K.Integrator.user(UF.HENON_HEILES, 2, 40, flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    qd0 = torch.from_numpy(q0.ravel().copy()).cuda()
    pd0 = torch.from_numpy(p0.ravel().copy()).cuda()
    qo = torch.empty(qh.size, dtype=torch.float64, device="cuda")
    po = torch.empty_like(qo)
    rc = K.irkgl16_integrate(dev.ctx, qd0, pd0, np.full(40, 0.2), np.full(40, 100, np.int64),
                             np.full(40, 10, np.int64), qo, po)
    assert rc == 0
    stream.synchronize()
    assert np.array_equal(qo.cpu().numpy(), qh) and np.array_equal(po.cpu().numpy(), ph)

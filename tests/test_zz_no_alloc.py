"""The allocation-free entry point (irkgl16_integrate_static, scratch in the
library's fixed device array) against the context path (irkgl16_create +
irkgl16_integrate with device pointers) on the same inputs: two calls in a
row, the second smaller, through the C ABI.  Both run the same kernels, so
frames, per-instance iteration counts and per-step counts must agree bit for
bit (the context path's chunks and promotions change only the schedule)."""
import ctypes as C

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


def batch(n, seed, max_steps, stride):
    """Uneven mix (gravity 3, 6, 16, 64 bodies; chains 32, 256, 1024 sites)
    with shortened step counts, plus one Kepler orbit."""
    insts = W.uneven_mix(n - 1, seed=seed, steps_range=(stride, max_steps), step_multiple=stride)
    kep = W.kepler_c1()
    kep["nsteps"] = max_steps
    insts.append(kep)
    return insts


def stats_struct(n, total_steps):
    st = K.irkgl16_stats()
    it = np.zeros(n, np.int64)
    ss = np.zeros(n, np.int32)
    si = np.zeros(max(total_steps, 1), np.uint8)
    st.inst_iterations = it.ctypes.data_as(C.POINTER(C.c_int64))
    st.inst_status = ss.ctypes.data_as(C.POINTER(C.c_int32))
    st.step_iters = si.ctypes.data_as(C.POINTER(C.c_uint8))
    return st, it, ss, si


def test_static_entry_point_matches_context_path_two_calls():
    import torch
    stream = torch.cuda.Stream()
    for n, seed, max_steps, stride, record in ((96, 11, 800, 50, True), (30, 12, 300, 100, False)):
        print(f"static entry point: {n} instances, up to {max_steps} steps, record={record}",
              flush=True)
        insts = batch(n, seed, max_steps, stride)
        problems = [prob(i) for i in insts]
        h = np.array([i["h"] for i in insts])
        ns = np.array([i["nsteps"] for i in insts], np.int64)
        sd = np.full(n, stride, np.int64)
        dq = np.array([i["n"] * i["d"] for i in insts], np.int64)
        total = int(np.sum(dq * (ns // sd + 1)))
        q0 = torch.from_numpy(np.concatenate([np.ravel(i["q"]) for i in insts])).cuda()
        p0 = torch.from_numpy(np.concatenate([np.ravel(i["p"]) for i in insts])).cuda()

        # context path
        qa = torch.empty(total, dtype=torch.float64, device="cuda")
        pa = torch.empty_like(qa)
        with K.Integrator(problems, record_iters=record, flags=K.IRKGL16_DEVICE_PTRS,
                          stream=stream) as ref:
            rc_a = K.irkgl16_integrate(ref.ctx, q0, p0, h, ns, sd, qa, pa)
            assert rc_a >= 0
            sa, ita, ssa, sia = stats_struct(n, int(ns.sum()))
            rc_a = K.irkgl16_last_stats(ref.ctx, sa)
        # allocation-free path; outputs pre-filled so unwritten frames show
        qb = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
        pb = torch.full((total,), float("nan"), dtype=torch.float64, device="cuda")
        torch.cuda.synchronize()
        sb, itb, ssb, sib = stats_struct(n, int(ns.sum()))
        rc_b = K.irkgl16_integrate_static(problems, q0, p0, h, ns, sd, qb, pb,
                                          record_iters=record, stream=stream, stats=sb)
        stream.synchronize()
        assert rc_b == rc_a and rc_b >= 0, (rc_a, rc_b)
        assert torch.equal(qa, qb) and torch.equal(pa, pb)
        assert np.array_equal(ita, itb) and np.array_equal(ssa, ssb)
        assert (sa.steps, sa.iterations, sa.nonconverged_steps, sa.max_k) == \
               (sb.steps, sb.iterations, sb.nonconverged_steps, sb.max_k)
        assert sb.steps == int(ns.sum())
        if record:
            assert np.array_equal(sia, sib) and sib.min() >= 1


def test_static_entry_point_rejects_oversized_calls():
    import torch
    q = torch.zeros(8, dtype=torch.float64, device="cuda")
    too_many = [dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)] * (K.IRKGL16_STATIC_MAX_INST + 1)
    assert K.irkgl16_integrate_static(too_many, q, q, 0.1, 10, 10, q, q) == K.IRKGL16_ESCRATCH
    too_big = [dict(kind=K.IRKGL16_CHAIN, n=1024, d=1, beta=1.0)] * 400
    assert K.irkgl16_integrate_static(too_big, q, q, 0.1, 10, 10, q, q) == K.IRKGL16_ESCRATCH

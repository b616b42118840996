#!/usr/bin/env python3
"""Throughput benchmark: batched FP64 IRKGL16 on the ensemble workload.

Workload (one bench step = one full integration call): 65,536 independent
6-body gravitational systems (central unit mass plus five planets, masses
U(1e-9, 1e-3), semi-major axes log-uniform in [5, 30], e <= 0.05,
inclination <= 2 deg, seeded), d = 3, G = 1, h = 1, 10^4 IRKGL16 steps each,
final state written (stride = 10^4).  Inputs and outputs are torch tensors
resident in HBM; the library enqueues on the bench's torch stream.

Printed JSON line (rank 0):
  value          instance-steps per second of the batched persistent kernel
  roofline       FP64 VALU roofline of the integration call: algorithmic flops
                 per call (per-instance-step formula with the kernels' own
                 iteration counts) over the HIP-event time of the call on its
                 stream -- all of its kernels: the small-system kernel's
                 chunks, the stage-parallel kernel's chunks for promoted
                 instances, the queue-order kernels
  cpu_baseline   the CPU oracle (OpenMP, all host cores) on a bounded sample
  plain          the plain one-launch-per-step-per-instance GPU form on a subset
  accuracy       fraction of instances whose relative energy error between the
                 first and last frame is <= 1e-12
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# The kernel classes of one integration call run concurrently on auxiliary
# streams, but HIP runs the kernels of streams that share a hardware queue one
# after another, and a process gets GPU_MAX_HW_QUEUES queues (4 by default,
# two of them taken by the default and the caller's streams).  With 8 the seven
# classes of the uneven mix overlap (7.3 s per call instead of 10.1-11.0 s);
# the ensemble call gains about 1 %.  Read when HIP initialises, so set here,
# before anything imports torch; a larger value already in the environment is
# kept.
try:
    _hwq = int(os.environ.get("GPU_MAX_HW_QUEUES", "4"))
except ValueError:
    _hwq = 4
if _hwq < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

METRIC = "FP64 IRKGL16 steps/s, batched vs plain, at rel err<=1e-12; p50/p99 solve latency"
N_INST, N_BODIES, D, NSTEPS, H = 65536, 6, 3, 10_000, 1.0
FP64_PEAK_TFLOPS = 78.6


def flops_per_iteration(n_bodies, dq):
    """Algorithmic flops of one fixed-point iteration of one instance: 8 stage
    force evaluations at 20 flops per ordered pair, plus the stage update and
    increment norm (21 flops per stage component)."""
    return 8 * 20 * n_bodies * (n_bodies - 1) + 8 * dq * 21


def flops_per_step_fixed(dq):
    """Initial guess (36 flops per stage component) and compensated update
    (50 flops per component), once per step."""
    return 8 * dq * 36 + 50 * dq


def gravity_energy(mass, q, p, G=1.0):
    """Total energy of many systems at once: mass (n, N), q/p (n, 3N)."""
    n = mass.shape[0]
    qq = q.reshape(n, -1, 3)
    pp = p.reshape(n, -1, 3)
    T = 0.5 * np.sum(np.sum(pp * pp, -1) / mass, -1)
    U = np.zeros(n)
    N = mass.shape[1]
    for a in range(N):
        for b in range(a + 1, N):
            r = np.sqrt(np.sum((qq[:, b] - qq[:, a]) ** 2, -1))
            U -= G * mass[:, a] * mass[:, b] / r
    return T + U


def cpu_baseline(sy, n_sample, nsteps):
    """Time the oracle (as it stands) on a seeded subset; instance-steps/s."""
    from oracle import oracle as orc
    sub = sy[:n_sample]
    specs = [orc.Spec(orc.GRAVITY, N_BODIES, D, mass=s["mass"]) for s in sub]
    q0 = np.concatenate([s["q"] for s in sub])
    p0 = np.concatenate([s["p"] for s in sub])
    orc.lib()
    t = time.perf_counter()
    r = orc.integrate_batch(specs, q0, p0, H, nsteps, nsteps)
    dt = time.perf_counter() - t
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return dict(value=n_sample * nsteps / dt, unit="instance-steps/s", cores=cores, kind="oracle",
                sample=f"{n_sample} instances x {nsteps} steps of the same workload "
                       f"({dt:.1f} s, OpenMP over instances, gcc -O2 strict IEEE)",
                rc=int(r["rc"]))


PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_2511_03655_amd", "csrc")


def source_digest(files):
    """sha256 over kernel source files (the ones a traffic measurement covers).
    C/C++ sources are hashed without comments and with whitespace runs
    collapsed, so that an edited comment does not retire a measurement of
    unchanged code; other files are hashed as they are."""
    import hashlib
    import re
    token = re.compile(r'"(?:\\.|[^"\\])*"|\'(?:\\.|[^\'\\])*\'|//[^\n]*|/\*.*?\*/', re.S)

    def code_only(text):
        text = token.sub(lambda m: "" if m.group(0).startswith("/") else m.group(0), text)
        return re.sub(r"\s+", " ", text).strip()

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            data = fh.read()
        if f.endswith((".h", ".hip", ".cpp")):
            data = code_only(data.decode()).encode()
        h.update(data)
    return h.hexdigest()


def profile_record(name, files):
    """Figures recorded in profiles/<name>.md by rocprofv3 runs (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE scaled by a copy-kernel calibration,
    issued FP64 flops per launch from the SQ instruction counters); empty if the
    profile is missing or the kernel sources changed since."""
    path = os.path.join(PROFILES, name + ".md")
    if not os.path.exists(path):
        return {}
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith(("traffic_bytes_per_launch", "source_sha256",
                                                "issued_fp64_flops_per_launch")):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.pop("source_sha256", None) != source_digest(files):
        return {}
    out = {}
    for k, v in rec.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def traffic_from_profile(name, files):
    """HBM bytes per launch recorded in profiles/<name>.md (None if missing or
    the kernel sources changed since)."""
    return profile_record(name, files).get("traffic_bytes_per_launch")


def copy_calibration():
    """A plain device copy of known size (the FETCH_SIZE / WRITE_SIZE scale)."""
    import torch
    n = 1 << 27  # doubles: 1 GiB per buffer
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def accuracy_sample(probs, mass, q0, p0, dq, nsteps, stream, K, n_glob=4096, n_loc=256,
                    loc_steps=1000):
    """Energy-error statistics on a sample of the same workload (eqs. DHglobmax and
    DHlocmax) and the fixed-point iteration histogram, outside the timed region.
    Global: the first n_glob systems over the full run, every 100 steps, with the
    iteration count of every step recorded.  Local: the first n_loc systems, every
    step of the first loc_steps."""
    import torch
    dev = torch.device("cuda:0")
    out = {}
    stride = 100
    nf = nsteps // stride + 1
    with K.Integrator(probs[:n_glob], record_iters=True) as it:
        qg, pg, st, rc = it.integrate(q0[:n_glob * dq], p0[:n_glob * dq], H, nsteps, stride)
    m = mass[:n_glob]
    Q, P = qg.reshape(n_glob, nf, dq), pg.reshape(n_glob, nf, dq)
    E = np.stack([gravity_energy(m, Q[:, f], P[:, f]) for f in range(nf)], 1)
    dglob = np.max(np.abs(E / E[:, :1] - 1), 1)
    k = st["step_iters"].astype(np.int64)
    hist = np.bincount(k, minlength=int(k.max()) + 1)
    out["DHglob_max"] = {"definition": "max over frames (every 100 steps) of |H_n - H_0|/|H_0| "
                                       "(eq. DHglobmax) per system",
                         "sample": f"first {n_glob} systems, full run",
                         "pass_frac_1e-12": float(np.mean(dglob <= 1e-12)),
                         "median": float(np.median(dglob)), "p90": float(np.percentile(dglob, 90)),
                         "max": float(dglob.max())}
    out["iterations_per_step_histogram"] = {
        "sample": f"first {n_glob} systems, every step of the full run",
        "counts_by_k": {str(i): int(c) for i, c in enumerate(hist) if c},
        "mean": float(k.mean())}
    with K.Integrator(probs[:n_loc]) as it:
        ql, pl, _, _ = it.integrate(q0[:n_loc * dq], p0[:n_loc * dq], H, loc_steps, 1)
    Q, P = ql.reshape(n_loc, loc_steps + 1, dq), pl.reshape(n_loc, loc_steps + 1, dq)
    m = mass[:n_loc]
    E = np.stack([gravity_energy(m, Q[:, f], P[:, f]) for f in range(loc_steps + 1)], 1)
    dloc = np.max(np.abs((E[:, 1:] - E[:, :-1]) / E[:, :-1]), 1)
    out["DHloc_max"] = {"definition": "max over steps of |H_n - H_{n-1}|/|H_{n-1}| "
                                      "(eq. DHlocmax) per system",
                        "sample": f"first {n_loc} systems, every step of the first "
                                  f"{loc_steps}",
                        "median": float(np.median(dloc)), "p90": float(np.percentile(dloc, 90)),
                        "max": float(dloc.max())}
    return out


def bulk_and_critical_path(probs, q0, p0, dq, nsteps, inst_it, stream, K, flops_fn):
    """The same call without the 1 % of systems that needed the most fixed-point
    iterations (close encounters), and the single most-iterating system alone:
    the bulk rate and the serial critical path of the call."""
    import torch
    dev = torch.device("cuda:0")
    n = len(probs)
    order = np.argsort(inst_it)
    keep = np.sort(order[: n - n // 100])
    pk = [probs[i] for i in keep]
    qk = np.concatenate([q0[i * dq:(i + 1) * dq] for i in keep])
    pkv = np.concatenate([p0[i * dq:(i + 1) * dq] for i in keep])
    res = {}
    with K.Integrator(pk, flags=K.IRKGL16_DEVICE_PTRS, stream=stream) as it:
        qd = torch.from_numpy(qk).to(dev)
        pd = torch.from_numpy(pkv).to(dev)
        qo = torch.empty(len(keep) * dq * 2, dtype=torch.float64, device=dev)
        po = torch.empty_like(qo)
        times = []
        for _ in range(2):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            K.irkgl16_integrate(it.ctx, qd, pd, np.full(len(keep), H),
                                np.full(len(keep), nsteps, np.int64),
                                np.full(len(keep), nsteps, np.int64), qo, po)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) / 1e3)
        st, _ = it.last_stats()
    dt = min(times)
    res["bulk"] = {"sample": f"the call without the {n - len(keep)} systems (1 %) with the "
                             "most fixed-point iterations",
                   "value": len(keep) * nsteps / dt, "unit": "instance-steps/s",
                   "seconds": dt, "mean_iterations_per_step": st["iterations"] / (len(keep) * nsteps),
                   "roofline_frac": flops_fn(st["iterations"], len(keep) * nsteps) / dt / 1e12
                   / FP64_PEAK_TFLOPS}
    j = int(order[-1])
    with K.Integrator([probs[j]]) as it:
        _, _, st1, _ = it.integrate(q0[j * dq:(j + 1) * dq], p0[j * dq:(j + 1) * dq], H, nsteps,
                                    nsteps)
    res["critical_path"] = {"sample": f"system {j} (most fixed-point iterations) alone",
                            "seconds": st1["device_ms"] / 1e3,
                            "mean_iterations_per_step": st1["iterations"] / nsteps}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ode-steps", type=int, default=NSTEPS)
    ap.add_argument("--instances", type=int, default=N_INST)
    ap.add_argument("--cpu-sample", type=int, default=16384)
    ap.add_argument("--cpu-steps", type=int, default=4000)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "henon", "sbh", "stages",
                             "explicit"])
    ap.add_argument("--rates", default="",
                    help="served stream: comma-separated subset of the rates 10,100,1000,10000")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload != "c2":
        print(json.dumps(OTHER_WORKLOADS[args.workload](args)))
        return

    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import workloads as W

    n_inst, nsteps = args.instances, args.ode_steps
    dq = N_BODIES * D
    sy = W.planetary_systems(n_inst, N_BODIES)
    mass = np.stack([s["mass"] for s in sy])
    q0 = np.concatenate([s["q"] for s in sy])
    p0 = np.concatenate([s["p"] for s in sy])
    probs = [dict(kind=K.IRKGL16_GRAVITY, n=N_BODIES, d=D, mass=s["mass"], G=1.0, eps=0.0)
             for s in sy]

    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    integ = K.Integrator(probs, flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    q0_d = torch.from_numpy(q0).to(dev)
    p0_d = torch.from_numpy(p0).to(dev)
    q_out = torch.empty(n_inst * dq * 2, dtype=torch.float64, device=dev)
    p_out = torch.empty_like(q_out)
    torch.cuda.synchronize()

    def call():
        rc = K.irkgl16_integrate(integ.ctx, q0_d, p0_d, np.full(n_inst, H),
                                 np.full(n_inst, nsteps, np.int64),
                                 np.full(n_inst, nsteps, np.int64), q_out, p_out)
        if rc < 0:
            raise K.IRKGL16Error(rc, "irkgl16_integrate")

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record(stream)
        call()
        e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kernel_ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    stats, rc = integ.last_stats()

    inst_steps = n_inst * nsteps
    value = args.steps * inst_steps / elapsed
    iters = int(stats["iterations"])

    def call_flops(iterations, instance_steps):
        return iterations * flops_per_iteration(N_BODIES, dq) + \
            instance_steps * flops_per_step_fixed(dq)

    flops = call_flops(iters, inst_steps)
    avg_s = float(np.mean(kernel_ms)) / 1e3
    achieved = flops / avg_s / 1e12
    tail = None
    if not args.no_plain:
        tail = bulk_and_critical_path(probs, q0, p0, dq, nsteps, stats["inst_iterations"],
                                      stream, K, call_flops)

    # accuracy gate on the last call's output frames (first and last)
    qo = q_out.cpu().numpy().reshape(n_inst, 2, dq)
    po = p_out.cpu().numpy().reshape(n_inst, 2, dq)
    E0 = gravity_energy(mass, qo[:, 0], po[:, 0])
    E1 = gravity_energy(mass, qo[:, 1], po[:, 1])
    dE = np.abs(E1 / E0 - 1)
    gate = float(np.mean(dE <= 1e-12))
    inst_it = stats["inst_iterations"]
    accuracy = {"gate": "relative energy error first->last frame <= 1e-12 (every instance)",
                "pass_frac": gate, "median_dE": float(np.median(dE)),
                "steps_at_max_iter": int(stats["nonconverged_steps"]),
                "instances_with_capped_steps": int(np.sum(stats["inst_status"] ==
                                                          K.IRKGL16_ENOCONV))}
    if not args.no_plain:
        accuracy.update(accuracy_sample(probs, mass, q0, p0, dq, nsteps, stream, K))

    plain = None
    if not args.no_plain:
        n_p, s_p = 1024, 1000
        pi = K.Integrator(probs[:n_p], flags=K.IRKGL16_PLAIN)
        pi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, 20, 20)  # warm-up
        t = time.perf_counter()
        _, _, pst, _ = pi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, s_p, s_p)
        dtp = time.perf_counter() - t
        gi = K.Integrator(probs[:n_p], flags=K.IRKGL16_PLAIN | K.IRKGL16_GRAPH)
        gi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, 20, 20)
        t = time.perf_counter()
        gi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, s_p, s_p)
        dtg = time.perf_counter() - t
        bi = K.Integrator(probs[:n_p])
        bi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, 20, 20)
        t = time.perf_counter()
        bi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, s_p, s_p)
        dtb = time.perf_counter() - t
        plain = dict(value=n_p * s_p / dtp, unit="instance-steps/s",
                     sample=f"{n_p} instances x {s_p} steps, one launch per step per instance",
                     graph_replay=n_p * s_p / dtg,
                     batched_same_sample=n_p * s_p / dtb,
                     full_batch_speedup=value / (n_p * s_p / dtp))
        pi.close()
        gi.close()
        bi.close()

    repro = None
    if not args.no_plain:
        # reproducible (bit-identical to the strict-IEEE reference order) mode, one call
        ri = K.Integrator(probs, flags=K.IRKGL16_DEVICE_PTRS | K.IRKGL16_REPRODUCIBLE,
                          stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        rc_r = K.irkgl16_integrate(ri.ctx, q0_d, p0_d, np.full(n_inst, H),
                                   np.full(n_inst, nsteps, np.int64),
                                   np.full(n_inst, nsteps, np.int64), q_out, p_out)
        torch.cuda.synchronize()
        dtr = time.perf_counter() - t
        repro = dict(value=inst_steps / dtr, unit="instance-steps/s", rc=int(rc_r),
                     sample="full workload, one call, IRKGL16_REPRODUCIBLE")
        ri.close()

    served = None
    if not args.no_served:
        # bounded sample of the served stream: Poisson arrivals of the uneven mix
        from paper_2511_03655_amd import serve
        reqs = W.poisson_requests(1000.0, 400, steps_range=(1e3, 1e4), stride=100,
                                  plummer_sizes=(64, 128))
        so = serve.run_stream(reqs, cap_bytes=8 << 30, slice_steps=1000)
        served = dict(rate_per_s=1000.0, requests=len(reqs), p50_latency_s=so["p50_s"],
                      p99_latency_s=so["p99_s"], steps_per_s=so["steps_per_s"],
                      sample="400 Poisson requests at 1000/s from the uneven mix and Plummer "
                             "clusters of 64-128 bodies, 1e3..1e4 steps, output every 100 steps, "
                             "time slices of 1000 steps")

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sy, min(args.cpu_sample, n_inst), args.cpu_steps)

    prof = profile_record("small_kernel_c2_65536x6body",
                          ["k_small.hip", "small_kernel.h", "device_common.h", "k_prepare.hip",
                           "k_stage.hip", "runtime.hip"])
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "instance-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded planetary systems shaped like the outer Solar System problem)",
        "config": {"workload": f"{n_inst} x 6-body gravitational systems, d=3, h=1, "
                               f"{nsteps} IRKGL16 steps each, final state output",
                   "n_inst": n_inst, "n_bodies": N_BODIES, "ode_steps": nsteps, "h": H,
                   "parallelism": "single GPU"},
        "force_evals_per_s": 8 * iters * args.steps / elapsed,
        "mean_iterations_per_step": iters / inst_steps,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                     "traffic": prof.get("traffic_bytes_per_launch"),
                     "traffic_GBps": (prof["traffic_bytes_per_launch"] / avg_s / 1e9
                                      if "traffic_bytes_per_launch" in prof else None),
                     "issued": ({"flops_per_launch": prof["issued_fp64_flops_per_launch"],
                                 "achieved": prof["issued_fp64_flops_per_launch"] / avg_s / 1e12,
                                 "frac": prof["issued_fp64_flops_per_launch"] / avg_s / 1e12
                                 / FP64_PEAK_TFLOPS,
                                 "source": "rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes, "
                                           "profiles/small_kernel_c2_65536x6body.md"}
                                if "issued_fp64_flops_per_launch" in prof else None),
                     "kernel": "integration call: small_kernel<gravity, 6 bodies, d=3> in "
                               "chunks, stage_kernel for promoted instances, queue-order kernels",
                     "kernel_ms": float(np.mean(kernel_ms)),
                     "algorithmic_flops_per_launch": flops},
        "accuracy": accuracy,
        "stragglers": tail,
        "plain": plain,
        "reproducible": repro,
        "served": served,
        "cpu_baseline": cpu,
        "status": rc,
    }
    print(json.dumps(out))
    integ.close()


# ---------------------------------------------------------------------------
# The other configurations (run with --workload; the default line is c2).

def _common(metric_unit, value, cfg, extra):
    out = {"metric": METRIC, "value": value, "unit": metric_unit, "n_gpus": 1,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic", "config": cfg}
    out.update(extra)
    return out


def _problem(inst):
    p = dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
             eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
    if inst.get("mass") is not None:
        p["mass"] = inst["mass"]
    return p


def _flops_inst_step(inst, k):
    """Algorithmic flops of one step with k iterations (same convention as c2)."""
    n, dq = inst["n"], inst["n"] * inst["d"]
    if inst["kind"] == 0:
        fg = 10
    elif inst["kind"] == 1:
        fg = 20 * n * (n - 1)
    else:
        fg = 6 * n
    return k * (8 * fg + 8 * dq * 21) + 8 * dq * 36 + 50 * dq


def _timed_gpu(integ, q0, p0, h, ns, sd, reps=1, ode=False):
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    dev = torch.device("cuda:0")
    q0d = torch.from_numpy(np.ascontiguousarray(q0)).to(dev)
    p0d = None if ode else torch.from_numpy(np.ascontiguousarray(p0)).to(dev)
    total = int(np.sum(integ.dq * (np.asarray(ns) // np.asarray(sd) + 1)))
    qo = torch.empty(total, dtype=torch.float64, device=dev)
    po = None if ode else torch.empty_like(qo)
    ones = np.ones(len(np.atleast_1d(ns)), np.int64)
    K.irkgl16_integrate(integ.ctx, q0d, p0d, h, ones, ones, qo, po)  # warm-up: one step
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        rc = K.irkgl16_integrate(integ.ctx, q0d, p0d, h, ns, sd, qo, po)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / reps
    st, rc2 = integ.last_stats()
    return dt, st, rc2, qo, po


def run_c1(args):
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import workloads as W
    from oracle import oracle as orc
    c1 = W.kepler_c1()
    n = c1["nsteps"]
    stream = torch.cuda.Stream()
    prob = [dict(kind=0, n=1, d=2, G=1.0)]
    integ = K.Integrator(prob, flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    dt, st, rc, qo, po = _timed_gpu(integ, c1["q"], c1["p"], np.array([c1["h"]]),
                                    np.array([n]), np.array([1]), reps=3)
    plain = K.Integrator(prob, flags=K.IRKGL16_PLAIN)
    t = time.perf_counter()
    plain.integrate(c1["q"], c1["p"], c1["h"], 2000, 2000)
    dtp = (time.perf_counter() - t) / 2000
    integ.close()
    plain.close()
    sp = orc.Spec(orc.KEPLER, 1, 2, G=1.0)
    t = time.perf_counter()
    r = orc.integrate(sp, c1["q"], c1["p"], c1["h"], n, 1)
    dtc = time.perf_counter() - t
    q = qo.cpu().numpy().reshape(-1, 2)
    rel = float(np.max(np.abs(q - r["q"])) / np.max(np.abs(r["q"])))
    return _common("steps/s", n / dt,
                   {"workload": "planar Kepler a=1 e=0.6, 1 instance, h=2pi/128, 1e4 steps, "
                                "every step output"},
                   {"ms_per_step": dt * 1e3, "mean_iterations_per_step": st["iterations"] / n,
                    "max_rel_diff_vs_oracle_all_frames": rel,
                    "plain": {"value": 1.0 / dtp, "unit": "steps/s",
                              "sample": "2000 steps, one launch per step"},
                    "cpu_baseline": {"value": n / dtc, "unit": "steps/s", "cores": 1,
                                     "kind": "oracle", "sample": "the full 1e4 steps"}})


def run_c3(args):
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import workloads as W
    from oracle import oracle as orc
    inst = W.plummer(2048)
    n = 1000
    stream = torch.cuda.Stream()
    integ = K.Integrator([_problem(inst)], flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    dt, st, rc, qo, po = _timed_gpu(integ, inst["q"], inst["p"], np.array([inst["h"]]),
                                    np.array([n]), np.array([n]), reps=2)
    k = st["iterations"] / n
    flops = st["iterations"] * (8 * 20 * 2048 * 2047 + 8 * 6144 * 21) + n * (8 * 6144 * 36 + 50 * 6144)
    pairs = st["iterations"] * 8 * 2048 * 2047
    plain = K.Integrator([_problem(inst)], flags=K.IRKGL16_PLAIN)
    t = time.perf_counter()
    plain.integrate(inst["q"], inst["p"], inst["h"], 50, 50)
    dtp = (time.perf_counter() - t) / 50
    integ.close()
    plain.close()
    # bytes and issued FP64 flops per 1000-step launch (the call timed here)
    prof = profile_record("large_kernel_c3_plummer2048",
                          ["k_large.hip", "device_common.h", "pair_weight.h"])
    c3_traffic = prof.get("traffic_bytes_per_launch")
    sp = orc.Spec(orc.GRAVITY, 2048, 3, mass=inst["mass"], eps=inst["eps"])
    t = time.perf_counter()
    orc.integrate(sp, inst["q"], inst["p"], inst["h"], 10, 10)
    dtc = (time.perf_counter() - t) / 10
    return _common("steps/s", n / dt,
                   {"workload": "Plummer N=2048, eps=1e-2, h=1e-3, 1e3 steps, final state"},
                   {"ms_per_step": dt / n * 1e3, "mean_iterations_per_step": k,
                    "pair_interactions_per_s": pairs / dt,
                    "roofline": {"bound": "alu", "achieved": flops / dt / 1e12,
                                 "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops / dt / 1e12 / FP64_PEAK_TFLOPS,
                                 "traffic": c3_traffic,
                                 "traffic_GBps": (c3_traffic / dt / 1e9
                                                  if c3_traffic else None),
                                 "issued": ({"flops_per_launch":
                                                 prof["issued_fp64_flops_per_launch"],
                                             "achieved": prof["issued_fp64_flops_per_launch"]
                                                 / dt / 1e12,
                                             "frac": prof["issued_fp64_flops_per_launch"]
                                                 / dt / 1e12 / FP64_PEAK_TFLOPS,
                                             "source": "rocprofv3 SQ_INSTS_VALU_FLOPS_FP64 x 64 "
                                                       "lanes, profiles/large_kernel_c3_"
                                                       "plummer2048.md"}
                                            if "issued_fp64_flops_per_launch" in prof else None),
                                 "kernel": "large_kernel (cooperative, whole GPU)"},
                    "plain": {"value": 1.0 / dtp, "unit": "steps/s",
                              "sample": "50 steps, one launch per step"},
                    "cpu_baseline": {"value": 1.0 / dtc, "unit": "steps/s", "cores": 1,
                                     "kind": "oracle", "sample": "10 steps (single instance, "
                                                                 "one thread)"}})


def run_c4(args):
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import workloads as W
    from oracle import oracle as orc
    t0 = time.perf_counter()
    mix = W.uneven_mix(4096)
    print(f"c4: generated {len(mix)} instances in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    probs = [_problem(m) for m in mix]
    h = np.array([m["h"] for m in mix])
    ns = np.array([m["nsteps"] for m in mix], np.int64)
    q0 = np.concatenate([m["q"] for m in mix])
    p0 = np.concatenate([m["p"] for m in mix])
    stream = torch.cuda.Stream()
    integ = K.Integrator(probs, flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    dt, st, rc, qo, po = _timed_gpu(integ, q0, p0, h, ns, ns, reps=1)
    print(f"c4: batched run {dt:.2f} s", file=sys.stderr, flush=True)
    its = st["inst_iterations"]
    flops = sum(_flops_inst_step(m, it / m["nsteps"]) * m["nsteps"] for m, it in zip(mix, its))
    total_steps = int(ns.sum())
    # plain form on a sample: 2 instances of every class, 100 steps each
    sample = []
    seen = {}
    for i, m in enumerate(mix):
        if seen.get(m["cls"], 0) < 2:
            seen[m["cls"]] = seen.get(m["cls"], 0) + 1
            sample.append(i)
    pp = [probs[i] for i in sample]
    pq = np.concatenate([mix[i]["q"] for i in sample])
    pv = np.concatenate([mix[i]["p"] for i in sample])
    plain = K.Integrator(pp, flags=K.IRKGL16_PLAIN)
    t = time.perf_counter()
    plain.integrate(pq, pv, h[sample], 100, 100)
    dtp = time.perf_counter() - t
    bat = K.Integrator(pp)
    bat.integrate(pq, pv, h[sample], 20, 20)
    t = time.perf_counter()
    bat.integrate(pq, pv, h[sample], 100, 100)
    dtb = time.perf_counter() - t
    integ.close()
    plain.close()
    bat.close()
    # serial critical path: the call cannot end before its slowest instance,
    # and one instance runs on one CU (or one slot); the three instances with
    # the most work (iterations x per-iteration cost) timed alone
    cost = np.array([it * (m["n"] ** 2 if m["kind"] == 1 else m["n"]) for m, it in zip(mix, its)])
    crit = []
    for i in np.argsort(cost)[-3:][::-1]:
        m = mix[int(i)]
        with K.Integrator([probs[int(i)]]) as one:
            _, _, s1, _ = one.integrate(m["q"], m["p"], m["h"], m["nsteps"], m["nsteps"])
        crit.append({"instance": int(i), "class": m["cls"], "steps": int(m["nsteps"]),
                     "mean_iterations_per_step": s1["iterations"] / m["nsteps"],
                     "seconds_alone": s1["device_ms"] / 1e3})
    print(f"c4: critical path {max(c['seconds_alone'] for c in crit):.2f} s", file=sys.stderr,
          flush=True)
    c4_traffic = traffic_from_profile("uneven_mix_c4_4096",
                                      ["k_small.hip", "small_kernel.h", "k_stage.hip", "k_wg.hip",
                                       "k_prepare.hip", "device_common.h", "runtime.hip",
                                       "pair_weight.h"])
    specs = [orc.Spec(mix[i]["kind"], mix[i]["n"], mix[i]["d"], mass=mix[i].get("mass"),
                      G=mix[i].get("G", 1.0), beta=mix[i].get("beta", 0.0)) for i in sample]
    t = time.perf_counter()
    orc.integrate_batch(specs, pq, pv, h[sample], 100, 100)
    dtc = time.perf_counter() - t
    return _common("instance-steps/s", total_steps / dt,
                   {"workload": "4096 uneven instances: gravity 3/6/16/64 bodies and FPU-beta "
                                "chains 32/256/1024 sites, per-instance h, 1e3..1e5 steps"},
                   {"seconds": dt, "instance_steps": total_steps,
                    "roofline": {"bound": "alu", "achieved": flops / dt / 1e12,
                                 "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops / dt / 1e12 / FP64_PEAK_TFLOPS,
                                 "traffic": c4_traffic,
                                 "traffic_GBps": c4_traffic / dt / 1e9 if c4_traffic else None},
                    "critical_path": {"instances_alone": crit,
                                      "call_over_longest_alone":
                                          dt / max(c["seconds_alone"] for c in crit)},
                    "plain": {"value": len(sample) * 100 / dtp, "unit": "instance-steps/s",
                              "batched_same_sample": len(sample) * 100 / dtb,
                              "sample": f"{len(sample)} instances (2 per class) x 100 steps"},
                    "cpu_baseline": {"value": len(sample) * 100 / dtc, "unit": "instance-steps/s",
                                     "cores": int(os.environ.get("OMP_NUM_THREADS",
                                                                 os.cpu_count() or 1)),
                                     "kind": "oracle", "sample": "same 14 instances x 100 steps"}})


def _served_row(rate, nreq, so):
    st = so["server"]
    slices = max(st["slices"], 1)
    return dict(rate_per_s=rate, requests=nreq, completed=so["completed"],
                cancelled=so["cancelled"], cancelled_mean_progress=so["cancelled_progress"],
                p50_latency_s=so["p50_s"], p90_latency_s=so["p90_s"],
                p99_latency_s=so["p99_s"], max_latency_s=so["max_s"],
                steps_per_s=so["steps_per_s"], wall_s=so["wall_s"],
                slices=st["slices"], max_resident=st["max_resident"],
                slice_wall_ms=1e3 * st["slice_wall_s"] / slices,
                slice_device_ms=1e3 * st["slice_device_s"] / slices,
                slice_host_overhead_ms=1e3 * (st["slice_wall_s"] - st["slice_device_s"]) / slices)


def run_c5(args):
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import serve
    from paper_2511_03655_amd import workloads as W
    rows = []
    sat = None
    sweep = ((10.0, 60), (100.0, 300), (1000.0, 600), (10000.0, 1000))
    if args.rates:
        keep = {float(x) for x in args.rates.split(",")}
        sweep = tuple(r for r in sweep if r[0] in keep)
    for rate, nreq in sweep:
        reqs = W.poisson_requests(rate, nreq, steps_range=(1e3, 1e5), stride=100,
                                  plummer_sizes=(64, 128, 256))
        so = serve.run_stream(reqs, cap_bytes=64 << 30, slice_steps=1000)
        print(f"c5: rate {rate}/s done in {so['wall_s']:.1f} s", file=sys.stderr, flush=True)
        rows.append(_served_row(rate, nreq, so))
        sat = reqs
    # the last (most saturated) sample of the sweep as one batched call
    probs = [_problem(i) for _, i in sat]
    ns = np.array([i["nsteps"] for _, i in sat], np.int64)
    q0 = np.concatenate([i["q"] for _, i in sat])
    p0 = np.concatenate([i["p"] for _, i in sat])
    h = np.array([i["h"] for _, i in sat])
    with K.Integrator(probs) as integ:
        t = time.perf_counter()
        _, _, bst, _ = integ.integrate(q0, p0, h, ns, np.full(len(sat), 100, np.int64))
        dtb = time.perf_counter() - t
    batched = {"value": float(ns.sum()) / dtb, "unit": "instance-steps/s", "seconds": dtb,
               "sample": f"the {len(sat)} requests of the last row in one irkgl16_integrate "
                         "call (host buffers, frames every 100 steps)"}
    print(f"c5: same requests batched in {dtb:.1f} s", file=sys.stderr, flush=True)
    # the configured distribution at one rate: steps 1e3..1e6, clusters up to
    # 512 bodies, 120 s of arrivals; requests still running then are cancelled
    conf = None
    if not args.no_plain:
        reqs = W.poisson_requests(10.0, 1200, steps_range=(1e3, 1e6), stride=100,
                                  plummer_sizes=(64, 128, 256, 512))
        so = serve.run_stream(reqs, cap_bytes=64 << 30, slice_steps=1000, duration_s=120.0)
        conf = _served_row(10.0, len([r for r in reqs if r[0] <= 120.0]), so)
        conf["sample"] = ("Poisson 10/s for 120 s; uneven-mix requests and Plummer clusters "
                          "of 64-512 bodies, 1e3..1e6 steps, output every 100 steps, 64 GB cap; "
                          "latencies over the requests completed within the window, the rest "
                          "cancelled at 120 s")
        print(f"c5: configured stream {so['completed']} completed, {so['cancelled']} cancelled",
              file=sys.stderr, flush=True)
    best = max(r["steps_per_s"] for r in rows)
    return _common("instance-steps/s", best,
                   {"workload": "served Poisson stream of the uneven mix plus Plummer clusters "
                                "(64-256 bodies), 1e3..1e5 steps, output every 100 steps, "
                                "64 GB admission cap, slices of 1000 steps"},
                   {"rates": rows, "batched_same_requests": batched,
                    "served_over_batched": rows[-1]["steps_per_s"] / batched["value"],
                    "configured_distribution": conf})


def run_henon(args):
    """Henon-Heiles ensemble through the run-time compiled user force."""
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import user_forces as UF
    from paper_2511_03655_amd import workloads as W
    from oracle import oracle as orc
    n_inst, nsteps, h = 262144, 10_000, 2 * np.pi / 64
    q0, p0 = W.henon_heiles_ensemble(n_inst)
    q0, p0 = q0.ravel(), p0.ravel()
    stream = torch.cuda.Stream()
    t = time.perf_counter()
    integ = K.Integrator.user(UF.HENON_HEILES, 2, n_inst, flags=K.IRKGL16_DEVICE_PTRS,
                              stream=stream)
    t_compile = time.perf_counter() - t
    ns = np.full(n_inst, nsteps, np.int64)
    dt, st, rc, qo, po = _timed_gpu(integ, q0, p0, np.full(n_inst, h), ns, ns, reps=2)
    inst_steps = n_inst * nsteps
    k = st["iterations"] / inst_steps
    # 8 flops per stage force evaluation (two components), the rest as c2's convention
    flops = st["iterations"] * (8 * 8 + 8 * 2 * 21) + inst_steps * (8 * 2 * 36 + 50 * 2)
    kern_s = st["device_ms"] / 1e3
    q = qo.cpu().numpy().reshape(n_inst, 2, 2)
    p = po.cpu().numpy().reshape(n_inst, 2, 2)

    def hh_energy(q, p):
        return 0.5 * (p ** 2).sum(-1) + 0.5 * (q ** 2).sum(-1) + q[..., 0] ** 2 * q[..., 1] \
            - q[..., 1] ** 3 / 3

    dE = np.abs(hh_energy(q[:, 1], p[:, 1]) / hh_energy(q[:, 0], p[:, 0]) - 1)
    n_p, s_p = 64, 200
    plain = K.Integrator.user(UF.HENON_HEILES, 2, n_p, flags=K.IRKGL16_PLAIN)
    plain.integrate(q0[:2 * n_p], p0[:2 * n_p], h, 20, 20)
    t = time.perf_counter()
    plain.integrate(q0[:2 * n_p], p0[:2 * n_p], h, s_p, s_p)
    dtp = time.perf_counter() - t
    integ.close()
    plain.close()
    cpu = None
    if not args.no_cpu:
        n_c, s_c = 65536, 8000
        specs = [orc.Spec(orc.HENON, 1, 2)] * n_c
        orc.lib()
        t = time.perf_counter()
        orc.integrate_batch(specs, q0[:2 * n_c], p0[:2 * n_c], h, s_c, s_c)
        dtc = time.perf_counter() - t
        cpu = {"value": n_c * s_c / dtc, "unit": "instance-steps/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"{n_c} instances x {s_c} steps ({dtc:.1f} s, OpenMP over instances)"}
    return _common("instance-steps/s", inst_steps / dt,
                   {"workload": f"{n_inst} Henon-Heiles orbits near q2=0.3, p2=0.2 at H=1/12, "
                                f"h=2pi/64, {nsteps} steps, final state; force given as device "
                                "source and compiled at run time"},
                   {"seconds": dt, "compile_and_create_s": t_compile,
                    "mean_iterations_per_step": k,
                    "roofline": {"bound": "alu", "achieved": flops / kern_s / 1e12,
                                 "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops / kern_s / 1e12 / FP64_PEAK_TFLOPS,
                                 "traffic": traffic_from_profile(
                                     "lane_kernel_henon_262144",
                                     ["lane_kernel.h", "device_common.h", "k_prepare.hip",
                                      "user_force.cpp", "../user_forces.py"]),
                                 "kernel": "lane_kernel<user, Dq=2> (hiprtc)",
                                 "kernel_ms": st["device_ms"]},
                    "accuracy": {"gate": "relative energy error first->last frame <= 1e-12",
                                 "pass_frac": float(np.mean(dE <= 1e-12)),
                                 "median_dE": float(np.median(dE))},
                    "plain": {"value": n_p * s_p / dtp, "unit": "instance-steps/s",
                              "sample": f"{n_p} instances x {s_p} steps, one launch per step "
                                        "per instance"},
                    "cpu_baseline": cpu})


def run_sbh(args):
    """First-order form: charged particles near a Schwarzschild black hole
    (eq. Ham_SBH), right-hand side compiled at run time."""
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import user_forces as UF
    from paper_2511_03655_amd import workloads as W
    from oracle import oracle as orc
    n_inst, nsteps, h = 65536, 10_000, 2.0
    Y0 = W.schwarzschild_ensemble(n_inst)
    prm = np.tile(W.SBH_PARAMS, (n_inst, 1))
    stream = torch.cuda.Stream()
    t = time.perf_counter()
    integ = K.Integrator.ode(UF.SCHWARZSCHILD_RHS, 4, n_inst, params=prm,
                             flags=K.IRKGL16_DEVICE_PTRS, stream=stream)
    t_compile = time.perf_counter() - t
    ns = np.full(n_inst, nsteps, np.int64)
    y0 = Y0.ravel()
    dt, st, rc, yo, _ = _timed_gpu(integ, y0, y0, np.full(n_inst, h), ns, ns, reps=2, ode=True)
    inst_steps = n_inst * nsteps
    k = st["iterations"] / inst_steps
    # 40 flops per right-hand-side evaluation (trigonometric calls, square
    # roots and divisions count 1), the rest by the per-component convention
    flops = st["iterations"] * (8 * 40 + 8 * 4 * 21) + inst_steps * (8 * 4 * 36 + 50 * 4)
    kern_s = st["device_ms"] / 1e3
    y = yo.cpu().numpy().reshape(n_inst, 2, 4)
    E, L, b = W.SBH_PARAMS

    def energy(v):
        r, th, pr, pth = v[:, 0], v[:, 1], v[:, 2], v[:, 3]
        A = 1 - 2 / r
        u = r * r * np.sin(th) ** 2
        return 0.5 * A * pr * pr - 0.5 * E * E / A + pth * pth / (2 * r * r) + \
            (L - 0.5 * b * u) ** 2 / (2 * u)

    dE = np.abs(energy(y[:, 1]) - energy(y[:, 0])) / 0.5
    n_p, s_p = 64, 200
    plain = K.Integrator.ode(UF.SCHWARZSCHILD_RHS, 4, n_p, params=prm[:n_p],
                             flags=K.IRKGL16_PLAIN)
    plain.integrate(y0[:4 * n_p], None, h, 20, 20)
    t = time.perf_counter()
    plain.integrate(y0[:4 * n_p], None, h, s_p, s_p)
    dtp = time.perf_counter() - t
    integ.close()
    plain.close()
    cpu = None
    if not args.no_cpu:
        n_c, s_c = 65536, 5000
        spec = orc.Spec(orc.ODE_SBH, 1, 4, G=E, eps=L, beta=b)
        orc.lib()
        t = time.perf_counter()
        orc.integrate_ode_batch([spec] * n_c, y0[:4 * n_c], h, s_c, s_c)
        dtc = time.perf_counter() - t
        cpu = {"value": n_c * s_c / dtc, "unit": "instance-steps/s",
               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
               "kind": "oracle",
               "sample": f"{n_c} instances x {s_c} steps ({dtc:.1f} s, OpenMP over instances)"}
    return _common("instance-steps/s", inst_steps / dt,
                   {"workload": f"{n_inst} Schwarzschild-black-hole orbits (E=0.995, L=4.6, "
                                f"beta=8.9e-4, r0 in [10.5, 11.5], H=-1/2), first-order form, "
                                f"h={h}, {nsteps} steps, final state; right-hand side given as "
                                "device source and compiled at run time"},
                   {"seconds": dt, "compile_and_create_s": t_compile,
                    "mean_iterations_per_step": k,
                    "roofline": {"bound": "alu", "achieved": flops / kern_s / 1e12,
                                 "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": flops / kern_s / 1e12 / FP64_PEAK_TFLOPS,
                                 "traffic": None,
                                 "kernel": "lane_kernel<user ODE, D=4> (hiprtc)",
                                 "kernel_ms": st["device_ms"]},
                    "accuracy": {"gate": "relative energy error first->last frame <= 1e-12",
                                 "pass_frac": float(np.mean(dE <= 1e-12)),
                                 "median_dE": float(np.median(dE))},
                    "plain": {"value": n_p * s_p / dtp, "unit": "instance-steps/s",
                              "sample": f"{n_p} instances x {s_p} steps, one launch per step "
                                        "per instance"},
                    "cpu_baseline": cpu})


def run_stages(args):
    """Work-precision of the s-stage members (s = 2, 4, 6, 8) on a Henon-Heiles
    ensemble over a fixed time span: energy error against GPU time and force
    evaluations, for several step sizes per s (the comparison of the paper's
    section 5.2, here on the GPU)."""
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import user_forces as UF
    from paper_2511_03655_amd import workloads as W
    n_orb, periods, n_frames = 16384, 50, 50
    q0, p0 = W.henon_heiles_ensemble(n_orb)
    q0, p0 = q0.ravel(), p0.ravel()
    steps_per_period = {8: (4, 5, 6, 8, 12, 16, 32), 6: (6, 8, 10, 12, 16, 24, 32),
                        4: (16, 24, 32, 48, 64, 96), 2: (64, 128, 256, 512, 1024, 2048)}

    def energy(q, p):
        return 0.5 * (p ** 2).sum(-1) + 0.5 * (q ** 2).sum(-1) + q[..., 0] ** 2 * q[..., 1] \
            - q[..., 1] ** 3 / 3

    rows = {}
    best = None
    for s, nps in steps_per_period.items():
        stream = torch.cuda.Stream()
        integ = K.Integrator.user(UF.HENON_HEILES, 2, n_orb, flags=K.IRKGL16_DEVICE_PTRS,
                                  stream=stream, stages=s)
        out = []
        for m in nps:
            nsteps = periods * m
            h = 2 * np.pi / m
            ns = np.full(n_orb, nsteps, np.int64)
            sd = np.full(n_orb, nsteps // n_frames, np.int64)
            dt, st, rc, qo, po = _timed_gpu(integ, q0, p0, np.full(n_orb, h), ns, sd)
            q = qo.cpu().numpy().reshape(n_orb, n_frames + 1, 2)
            p = po.cpu().numpy().reshape(n_orb, n_frames + 1, 2)
            E = energy(q, p)
            per_orbit = np.max(np.abs(E / E[:, :1] - 1), axis=1)
            err = float(np.median(per_orbit)) if np.all(np.isfinite(per_orbit)) else float("inf")
            out.append({"h": h, "steps_per_orbit": nsteps, "energy_error": err,
                        "gpu_ms": st["device_ms"], "mean_iterations_per_step":
                        st["iterations"] / (n_orb * nsteps),
                        "force_evals_per_orbit": s * st["iterations"] / n_orb})
            print(f"stages: s={s} steps/period={m} err={err:.2e} {st['device_ms']:.1f} ms",
                  file=sys.stderr, flush=True)
        rows[s] = out
        integ.close()
    # cheapest run (GPU time) reaching each target precision, per s
    targets = (1e-10, 1e-12, 1e-13)
    fastest = {}
    for tgt in targets:
        cand = {s: min((r["gpu_ms"] for r in rs if r["energy_error"] <= tgt), default=None)
                for s, rs in rows.items()}
        reach = {s: v for s, v in cand.items() if v is not None}
        fastest[f"{tgt:.0e}"] = {"gpu_ms": cand, "fastest_s": min(reach, key=reach.get)
                                 if reach else None}
    r8 = rows[8][-1]
    value = n_orb * r8["steps_per_orbit"] / (r8["gpu_ms"] / 1e3)
    return _common("instance-steps/s", value,
                   {"workload": f"{n_orb} Henon-Heiles orbits near q2=0.3, p2=0.2 at H=1/12, "
                                f"{periods} periods (t = {periods} x 2 pi), s = 2, 4, 6, 8 "
                                "stages at several step sizes each; value: s = 8 at the "
                                "smallest step"},
                   {"work_precision": {str(s): rs for s, rs in rows.items()},
                    "error_measure": "median over orbits of max_t |H(t)/H(0) - 1| over "
                                     f"{n_frames} frames",
                    "cheapest_run_reaching": fastest})


def run_explicit(args):
    """IRKGL16 against the explicit symplectic baselines (Strang, SUZ90) on a
    Henon-Heiles ensemble: maximum local energy error (eq. DHlocmax) against
    GPU time and force evaluations, and the GPU time per force evaluation of
    IRKGL16 normalised by that of the explicit methods at the IRKGL16 step
    whose local energy error is closest to 1e-14 (the quantity of the paper's
    Table 1, there measured on one CPU core)."""
    import torch
    from paper_2511_03655_amd import irkgl16 as K
    from paper_2511_03655_amd import user_forces as UF
    from paper_2511_03655_amd import workloads as W
    n_orb, periods, n_err = 16384, 10, 256
    q0, p0 = W.henon_heiles_ensemble(n_orb)
    q0, p0 = q0.ravel(), p0.ravel()
    methods = {"IRKGL16": (0, 8, (3, 4, 5, 6, 8, 12)),
               "SUZ90": (K.IRKGL16_SUZ90, 5, (64, 128, 256, 512, 1024, 2048)),
               "Strang": (K.IRKGL16_STRANG, 1, (256, 1024, 4096, 16384))}

    def energy(q, p):
        return 0.5 * (p ** 2).sum(-1) + 0.5 * (q ** 2).sum(-1) + q[..., 0] ** 2 * q[..., 1] \
            - q[..., 1] ** 3 / 3

    rows = {}
    for name, (method, evals, nps) in methods.items():
        stream = torch.cuda.Stream()
        integ = K.Integrator.user(UF.HENON_HEILES, 2, n_orb, flags=K.IRKGL16_DEVICE_PTRS,
                                  stream=stream, method=method)
        probe = K.Integrator.user(UF.HENON_HEILES, 2, n_err, method=method)
        out = []
        for m in nps:
            h = 2 * np.pi / m
            nsteps = periods * m
            ns = np.full(n_orb, nsteps, np.int64)
            dt, st, rc, qo, po = _timed_gpu(integ, q0, p0, np.full(n_orb, h), ns, ns)
            f_evals = (8 * st["iterations"] if method == 0 else evals * n_orb * nsteps)
            # local energy error over one period, every step, on a subset
            qe, pe, ste, _ = probe.integrate(q0[:2 * n_err], p0[:2 * n_err], h, m, 1)
            E = energy(qe.reshape(n_err, m + 1, 2), pe.reshape(n_err, m + 1, 2))
            loc = np.max(np.abs(np.diff(E, axis=1) / E[:, :-1]), axis=1)
            out.append({"h": h, "steps_per_period": m, "local_energy_error": float(np.median(loc)),
                        "gpu_ms": st["device_ms"], "force_evals_per_orbit": f_evals / n_orb,
                        "gpu_ns_per_force_eval": st["device_ms"] * 1e6 / f_evals})
            print(f"explicit: {name} steps/period={m} err={np.median(loc):.2e} "
                  f"{st['device_ms']:.1f} ms", file=sys.stderr, flush=True)
        rows[name] = out
        integ.close()
        probe.close()
    ref = min(rows["IRKGL16"], key=lambda r: abs(np.log10(max(r["local_energy_error"], 1e-300))
                                                 + 14))
    per_eval_explicit = {n: float(np.median([r["gpu_ns_per_force_eval"] for r in rows[n]]))
                         for n in ("SUZ90", "Strang")}
    ratio = {n: ref["gpu_ns_per_force_eval"] / v for n, v in per_eval_explicit.items()}
    cheapest = {}
    for tgt in (1e-10, 1e-12, 1e-14):
        cheapest[f"{tgt:.0e}"] = {n: min((r["gpu_ms"] for r in rs
                                          if r["local_energy_error"] <= tgt), default=None)
                                  for n, rs in rows.items()}
    return _common("instance-steps/s", n_orb * periods * ref["steps_per_period"] /
                   (ref["gpu_ms"] / 1e3),
                   {"workload": f"{n_orb} Henon-Heiles orbits near q2=0.3, p2=0.2 at H=1/12, "
                                f"{periods} periods; IRKGL16 against Strang and SUZ90 "
                                "(user force compiled at run time); value: IRKGL16 at the step "
                                "with local energy error closest to 1e-14"},
                   {"work_precision": rows,
                    "error_measure": f"median over {n_err} orbits of max_n |H_n/H_(n-1) - 1| "
                                     "over one period (eq. DHlocmax)",
                    "irkgl16_reference_step": ref,
                    "gpu_fcn_ratio": {"irkgl16_over": ratio,
                                      "paper_table1_cpu_simd": 0.6,
                                      "paper_table1_cpu_seq": 2.5},
                    "cheapest_run_reaching_local_error": cheapest})


OTHER_WORKLOADS = {"c1": run_c1, "c3": run_c3, "c4": run_c4, "c5": run_c5, "henon": run_henon,
                   "sbh": run_sbh, "stages": run_stages, "explicit": run_explicit}


if __name__ == "__main__":
    main()

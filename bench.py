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
  roofline       FP64 VALU roofline of the integration kernel: algorithmic
                 flops per launch (per-instance-step formula with the kernel's
                 own iteration counts) over the HIP-event time of the launch
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
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

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
    flops = iters * flops_per_iteration(N_BODIES, dq) + inst_steps * flops_per_step_fixed(dq)
    avg_s = float(np.mean(kernel_ms)) / 1e3
    achieved = flops / avg_s / 1e12

    # accuracy gate on the last call's output frames (first and last)
    qo = q_out.cpu().numpy().reshape(n_inst, 2, dq)
    po = p_out.cpu().numpy().reshape(n_inst, 2, dq)
    E0 = gravity_energy(mass, qo[:, 0], po[:, 0])
    E1 = gravity_energy(mass, qo[:, 1], po[:, 1])
    dE = np.abs(E1 / E0 - 1)
    gate = float(np.mean(dE <= 1e-12))

    plain = None
    if not args.no_plain:
        n_p, s_p = 64, 200
        pi = K.Integrator(probs[:n_p], flags=K.IRKGL16_PLAIN)
        pi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, 20, 20)  # warm-up
        t = time.perf_counter()
        _, _, pst, _ = pi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, s_p, s_p)
        dtp = time.perf_counter() - t
        bi = K.Integrator(probs[:n_p])
        bi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, 20, 20)
        t = time.perf_counter()
        bi.integrate(q0[:n_p * dq], p0[:n_p * dq], H, s_p, s_p)
        dtb = time.perf_counter() - t
        plain = dict(value=n_p * s_p / dtp, unit="instance-steps/s",
                     sample=f"{n_p} instances x {s_p} steps, one launch per step per instance",
                     batched_same_sample=n_p * s_p / dtb,
                     full_batch_speedup=value / (n_p * s_p / dtp))
        pi.close()
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

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(sy, min(args.cpu_sample, n_inst), args.cpu_steps)

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
                     "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS, "traffic": None,
                     "kernel_ms": float(np.mean(kernel_ms)),
                     "algorithmic_flops_per_launch": flops},
        "accuracy": {"gate": "relative energy error first->last frame <= 1e-12",
                     "pass_frac": gate, "median_dE": float(np.median(dE))},
        "plain": plain,
        "reproducible": repro,
        "cpu_baseline": cpu,
        "status": rc,
    }
    print(json.dumps(out))
    integ.close()


if __name__ == "__main__":
    main()

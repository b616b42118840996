#!/usr/bin/env python3
"""Autotuner for the launch shapes of the integration kernels.

Tunes, on the GPU it runs on, the shapes that do not change results:

* ``wg/<kind>/<d>/<S>`` -- lanes per workgroup of the workgroup kernel for
  systems in slots of S lanes (systems per workgroup = block / S; gravity in
  the fast mode up to 256 bodies uses slots of 2 S lanes), timed on a batch of
  such systems;
* ``large/<n>`` -- sources staged per tile (128 or 256, split over the
  workgroup's 16 wavefronts) of the whole-GPU kernel for one system of up to
  n bodies;
* ``sched/max_chunks``, ``sched/promote_k10``, ``sched/evict_k10`` -- the
  schedule of a call with few-body gravitational systems (the classes that can
  promote run in chunks): the most chunks per call, and ten times the
  iterations per step from which an instance
  moves to the stage-parallel kernel between chunks or stops mid-chunk for it
  (0 = never), tuned one after another on the ensemble workload.

Each candidate is timed by creating a context whose tuning table holds only
that candidate (IRKGL16_TUNE_CACHE points at a temporary file); the fastest
candidate of every key is written to the cache (default: tune_cache.json next
to libirkgl16.so, which every context and server reads at creation).

    python -m paper_2511_03655_amd.autotune [--out PATH] [--quick]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import tempfile
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2511_03655_amd import irkgl16 as K  # noqa: E402
from paper_2511_03655_amd import workloads as W  # noqa: E402


def slot_width(n):
    """Slot width of the workgroup kernel for n bodies or sites."""
    if n <= 64:
        s = 8
        while s < n:
            s <<= 1
        return s
    return (n + 63) // 64 * 64


def problem(inst):
    p = dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
             eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
    if inst.get("mass") is not None:
        p["mass"] = inst["mass"]
    return p


def time_batch(insts, nsteps, cache_values, reps=2):
    """Seconds of one integration call of `insts` with the given tuning table
    (the best of `reps` timed calls)."""
    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        json.dump(cache_values, f)
        path = f.name
    old = os.environ.get("IRKGL16_TUNE_CACHE")
    os.environ["IRKGL16_TUNE_CACHE"] = path
    try:
        integ = K.Integrator([problem(m) for m in insts])
    finally:
        if old is None:
            del os.environ["IRKGL16_TUNE_CACHE"]
        else:
            os.environ["IRKGL16_TUNE_CACHE"] = old
        os.unlink(path)
    q0 = np.concatenate([m["q"] for m in insts])
    p0 = np.concatenate([m["p"] for m in insts])
    h = np.array([m["h"] for m in insts])
    integ.integrate(q0, p0, h, 2, 2)  # warm-up (code objects, allocations)
    best = float("inf")
    for _ in range(reps):
        t = time.perf_counter()
        integ.integrate(q0, p0, h, nsteps, nsteps)
        best = min(best, time.perf_counter() - t)
    integ.close()
    return best


SCHED_CANDIDATES = [("sched/max_chunks", [4, 6, 8, 12, 16]),
                    ("sched/promote_k10", [40, 50, 60, 80]),
                    ("sched/evict_k10", [80, 120, 160, 240])]


def tune_schedule(quick, base):
    """Coordinate descent over the schedule keys on the ensemble workload
    (6-body planetary systems, h = 1); `base` holds the keys chosen so far."""
    n_inst, nsteps = (16384, 4000) if quick else (65536, 10_000)
    sy = W.planetary_systems(n_inst, 6)
    for s in sy:
        s["h"] = 1.0
    chosen, report = {}, {}
    for key, cands in SCHED_CANDIDATES:
        times = {}
        for c in cands:
            table = dict(base)
            table.update(chosen)
            table[key] = c
            times[c] = time_batch(sy, nsteps, table)
            print(f"autotune {key} candidate {c}: {times[c] * 1e3:.2f} ms", flush=True)
        chosen[key] = min(times, key=times.get)
        report[key] = {str(c): round(t * 1e3, 3) for c, t in times.items()}
    return chosen, report


def cases(quick):
    """(key, candidates, instances, steps) to tune."""
    out = []
    n_inst = 128 if quick else 512
    for n in (32, 256, 1024):
        s = slot_width(n)
        cands = [b for b in (64, 128, 256, 512, 1024) if b >= s and b % s == 0]
        insts = [W.fpu_chain(n, seed=100 + i) for i in range(n_inst)]
        out.append((f"wg/2/1/{s}", cands, insts, 100 if quick else 300))
    for n in (256,):
        s = slot_width(n)
        # the fast mode gives gravity systems of up to 256 bodies two lanes per
        # body: the slot is twice the body slot (one candidate at 256 bodies)
        lanes = 2 * s if 2 * s <= 512 else s
        cands = [b for b in (256, 512) if b >= lanes and b % lanes == 0]
        insts = [W.plummer(n, seed=200 + i) for i in range(16 if quick else 64)]
        out.append((f"wg/1/3/{s}", cands, insts, 5 if quick else 20))
    # one call of the whole-GPU kernel lasts ~0.1 ms per step: 10^3 steps so that
    # launch and copy overheads do not hide a few per cent between tiles
    insts = [W.plummer(2048, seed=300)]
    out.append(("large/2048", [128, 256], insts, 200 if quick else 1000))
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=os.path.join(HERE, "tune_cache.json"))
    ap.add_argument("--quick", action="store_true", help="smaller timing batches")
    ap.add_argument("--no-schedule", action="store_true", help="launch shapes only")
    args = ap.parse_args()
    result, report = {}, {}
    for key, cands, insts, nsteps in cases(args.quick):
        if len(cands) == 1:
            result[key] = cands[0]
            continue
        times = {}
        for c in cands:
            times[c] = time_batch(insts, nsteps, {key: c}, reps=3)
            print(f"autotune {key} candidate {c}: {times[c] * 1e3:.2f} ms", flush=True)
        best = min(times, key=times.get)
        result[key] = best
        report[key] = {str(c): round(t * 1e3, 3) for c, t in times.items()}
    if not args.no_schedule:
        chosen, rep = tune_schedule(args.quick, result)
        result.update(chosen)
        report.update(rep)
    elif os.path.exists(args.out):  # launch shapes only: keep the schedule keys there
        with open(args.out) as f:
            result.update({k: v for k, v in json.load(f).items() if k.startswith("sched/")})
    with open(args.out, "w") as f:
        json.dump(result, f, indent=1, sort_keys=True)
    print(json.dumps({"cache": args.out, "chosen": result, "timings_ms": report}))


if __name__ == "__main__":
    main()

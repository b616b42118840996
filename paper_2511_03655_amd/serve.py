"""Open-loop Poisson client for the serving loop (served-stream workload).

Submits requests at their scheduled arrival times from one thread while
another consumes finished ones, then reports latency percentiles (submission to
completion) and throughput.  The arithmetic all happens in the library's
serving thread and kernels.
"""
from __future__ import annotations

import threading
import time

import numpy as np

from . import irkgl16 as K


def _problem(inst):
    p = dict(kind=inst["kind"], n=inst["n"], d=inst["d"], G=inst.get("G", 1.0),
             eps=inst.get("eps", 0.0), beta=inst.get("beta", 0.0))
    if inst.get("mass") is not None:
        p["mass"] = inst["mass"]
    return p


def run_stream(requests, cap_bytes=64 << 30, slice_steps=1000, keep_frames=False, flags=0,
               slice_ms=0.0, duration_s=None):
    """requests: list of (arrival_time_s, instance) with instance['nsteps'],
    ['stride'], ['h'].  With duration_s, requests arriving later are not sent
    and, once that time has passed, the ones not finished are cancelled (the
    latency statistics then cover the finished requests; the cancelled ones
    are counted with the fraction of their steps done).  Returns a dict with
    per-request latency, totals and the server's slice statistics."""
    if duration_s is not None:
        requests = [r for r in requests if r[0] <= duration_s]
    srv = K.Server(cap_bytes=cap_bytes, slice_steps=slice_steps, flags=flags, slice_ms=slice_ms)
    tickets = [None] * len(requests)
    results = [None] * len(requests)
    t0 = time.perf_counter()

    def producer():
        for i, (ta, inst) in enumerate(requests):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(_problem(inst), inst["q"], inst["p"], inst["h"],
                                    inst["nsteps"], inst["stride"])

    th = threading.Thread(target=producer)
    th.start()
    pending = set(range(len(requests)))
    cancelled_all = False
    while pending:
        progressed = False
        if duration_s is not None and not cancelled_all and time.perf_counter() - t0 > duration_s:
            th.join()
            for i in pending:
                srv.cancel(tickets[i])
            cancelled_all = True
        for i in list(pending):
            t = tickets[i]
            if t is not None and srv.poll(t):
                q, p, info, rc = srv.wait(t, keep_frames=keep_frames)
                results[i] = (q, p, info, rc)
                pending.discard(i)
                progressed = True
        if not progressed:
            time.sleep(0.0005)
    th.join()
    wall = time.perf_counter() - t0
    sstat = srv.stats()
    srv.close()
    done = [r for r in results if r[3] != K.IRKGL16_ECANCELED]
    lat = np.array([r[2]["done_s"] - r[2]["submit_s"] for r in done]) if done else np.zeros(1)
    steps = int(sum(r[2]["steps"] for r in results))
    canc = [(r[2]["steps"], inst["nsteps"]) for r, (_, inst) in zip(results, requests)
            if r[3] == K.IRKGL16_ECANCELED]
    return dict(latency_s=lat, p50_s=float(np.percentile(lat, 50)),
                p90_s=float(np.percentile(lat, 90)), p99_s=float(np.percentile(lat, 99)),
                max_s=float(lat.max()), wall_s=wall, steps=steps, steps_per_s=steps / wall,
                completed=len(done), cancelled=len(canc),
                cancelled_progress=(float(np.mean([a / b for a, b in canc])) if canc else None),
                server=sstat, results=results)

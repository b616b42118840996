"""Launch shapes from the tuning table (systems per workgroup, LDS tile size)
never change results: the same systems integrate to the same bits under every
candidate shape the autotuner may pick."""
import json
import os

import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K
from paper_2511_03655_amd import workloads as W

pytestmark = pytest.mark.gpu


def run_with(tmp_path, values, insts, nsteps, stride):
    path = tmp_path / f"tune_{abs(hash(json.dumps(values, sort_keys=True)))}.json"
    path.write_text(json.dumps(values))
    old = os.environ.get("IRKGL16_TUNE_CACHE")
    os.environ["IRKGL16_TUNE_CACHE"] = str(path)
    try:
        probs = []
        for m in insts:
            p = dict(kind=m["kind"], n=m["n"], d=m["d"], G=m.get("G", 1.0), eps=m.get("eps", 0.0),
                     beta=m.get("beta", 0.0))
            if m.get("mass") is not None:
                p["mass"] = m["mass"]
            probs.append(p)
        integ = K.Integrator(probs)
    finally:
        if old is None:
            del os.environ["IRKGL16_TUNE_CACHE"]
        else:
            os.environ["IRKGL16_TUNE_CACHE"] = old
    q0 = np.concatenate([m["q"] for m in insts])
    p0 = np.concatenate([m["p"] for m in insts])
    h = np.array([m["h"] for m in insts])
    return integ.integrate(q0, p0, h, nsteps, stride)


def test_workgroup_block_size_does_not_change_results(tmp_path):
    insts = [W.fpu_chain(32, seed=40 + i) for i in range(37)]
    ref = run_with(tmp_path, {}, insts, 60, 20)
    for block in (64, 128, 512, 1024):
        out = run_with(tmp_path, {"wg/2/1/32": block}, insts, 60, 20)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), block
        assert out[2]["iterations"] == ref[2]["iterations"]


def test_large_tile_does_not_change_results(tmp_path):
    insts = [W.plummer(1000, seed=41)]
    ref = run_with(tmp_path, {"large/1024": 256}, insts, 4, 2)
    out = run_with(tmp_path, {"large/1024": 128}, insts, 4, 2)
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


def test_invalid_table_entries_fall_back_to_defaults(tmp_path):
    insts = [W.fpu_chain(32, seed=42 + i) for i in range(5)]
    ref = run_with(tmp_path, {}, insts, 30, 30)
    out = run_with(tmp_path, {"wg/2/1/32": 96, "large/1024": 7}, insts, 30, 30)  # 96: not a slot multiple of 64
    assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1])


def test_schedule_keys_do_not_change_results(tmp_path):
    """Chunk count and the promotion and eviction thresholds decide only where
    and when a step runs: every candidate the autotuner may pick gives the
    same bits (planetary systems with close encounters, so that instances
    are promoted and evicted)."""
    insts = W.planetary_systems(600, 6, seed=77)
    for s in insts:
        s["h"] = 1.0
    ref = run_with(tmp_path, {"sched/promote_k10": 0, "sched/evict_k10": 0}, insts, 640, 320)
    for vals in ({}, {"sched/max_chunks": 4}, {"sched/max_chunks": 16, "sched/promote_k10": 40},
                 {"sched/max_chunks": 8, "sched/promote_k10": 20, "sched/evict_k10": 30}):
        out = run_with(tmp_path, vals, insts, 640, 320)
        assert np.array_equal(out[0], ref[0]) and np.array_equal(out[1], ref[1]), vals
        assert out[2]["iterations"] == ref[2]["iterations"], vals

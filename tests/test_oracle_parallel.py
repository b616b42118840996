"""The oracle spreads the targets of one large gravitational system over
threads (each target's pair sum keeps its ascending source order on one
thread); the results must not depend on the thread count."""
import numpy as np

from paper_2511_03655_amd import workloads as W


def test_parallel_targets_give_the_serial_bits(orc):
    inst = W.plummer(300, seed=31)   # above the oracle's threshold for threading
    sp = orc.Spec(orc.GRAVITY, 300, 3, mass=inst["mass"], G=inst["G"], eps=inst["eps"])
    out = {}
    try:
        for threads in (1, 4, 7):
            orc.set_threads(threads)
            r = orc.integrate(sp, inst["q"], inst["p"], inst["h"], 3, 1, want_iters=True)
            out[threads] = (orc.force(sp, inst["q"]), r["q"], r["p"], r["iters"])
    finally:
        orc.set_threads(0)
    for threads in (4, 7):
        for a, b in zip(out[1], out[threads]):
            assert np.array_equal(a, b), threads

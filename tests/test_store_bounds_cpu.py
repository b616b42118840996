"""Every global store of the batched kernels stays inside its instance's
allocation, and every output frame is written, over the launches of chunked,
one-launch and plain (one step per launch) calls with instances that stop at
a non-finite step or are evicted mid-chunk.  The index arithmetic is the
kernels' own (store_index.h); tests/store_bounds_check.cpp walks the launches
on the CPU, built with the host sanitizers."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_store_indices_stay_in_bounds(tmp_path):
    exe = str(tmp_path / "store_bounds_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", exe, os.path.join(HERE, "store_bounds_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert " 0 violations" in r.stdout

"""The serving loop's scheduling decisions (first-fit arena under the memory
cap, first-come-first-served admission, per-class slice budgets, staged and
harvested frame windows, cancellation between slices) driven by a fake
integrator on the CPU: tests/serve_sched_check.cpp, built with the host
sanitizers, uses the server's own helpers (serve_sched.h)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serving_schedule_with_a_fake_integrator(tmp_path):
    exe = str(tmp_path / "serve_sched_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-Werror",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-o", exe, os.path.join(HERE, "serve_sched_check.cpp")])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "0 failures" in r.stdout

"""The CPU suite under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with gcc's sanitizers and its pin tests run against that
build; the HIP library's host code (argument checks, layouts, the scratch-size
checks of the allocation-free entry point, the binding's marshalling) is
rebuilt with clang's sanitizers on the host side only (the gfx950 device code
is compiled as usual) and the C-ABI boundary tests run against it.  Each run
is a child process with the sanitizer runtime preloaded (the Python
interpreter itself is not instrumented); a report of either sanitizer fails
the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_PIN_TESTS = ["tests/test_oracle_pins.py", "tests/test_oracle_ode_pins.py",
                    "tests/test_oracle_split_pins.py", "tests/test_oracle_stages_pins.py",
                    "tests/test_oracle_parallel.py", "tests/test_oracle_tableau.py"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _child(tests, env_extra, timeout):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider", *tests], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=timeout)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, out
    return out


def _instrumented(lib):
    """The build calls into the sanitizer runtimes (it was compiled with them)."""
    syms = subprocess.run(["nm", "-D", "--undefined-only", lib], capture_output=True,
                          text=True).stdout
    return "__asan_report" in syms and "__ubsan_handle" in syms


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True,
                       text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import oracle as O
    lib = O.build(out=str(tmp_path / "liborc_san.so"),
                  extra_flags=("-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                               "-fno-omit-frame-pointer", "-g"))
    assert _instrumented(lib)
    out = _child(ORACLE_PIN_TESTS, {"LD_PRELOAD": f"{asan}:{ubsan}", "IRKGL16_ORACLE_LIB": lib},
                 timeout=900)
    assert " passed" in out


def _clang_asan_runtime():
    p = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True).stdout.strip()
    if os.path.isabs(p) and os.path.exists(p):
        return p
    p = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-runtime-dir"], capture_output=True,
                       text=True).stdout.strip()
    cand = os.path.join(p, "libclang_rt.asan.so")
    return cand if os.path.exists(cand) else None


def test_host_runtime_under_asan_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    if not rt:
        pytest.skip("clang sanitizer runtime not installed")
    sys.path.insert(0, ROOT)
    from paper_2511_03655_amd import build as B
    lib = B.build(verbose=False, out=str(tmp_path / "libirkgl16_san.so"),
                  objdir=str(tmp_path / "obj"),
                  host_flags=("-fsanitize=address", "-fsanitize=undefined",
                              "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                              "-shared-libasan"))
    assert _instrumented(lib)
    out = _child(["tests/test_boundary_cpu.py"], {"LD_PRELOAD": rt, "IRKGL16_LIB": lib},
                 timeout=900)
    assert " passed" in out

"""C-ABI boundary checks that need no GPU: the library loads, exports every
symbol the header declares, validates arguments and reports a missing device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2511_03655_amd import irkgl16 as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "irkgl16.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(irkgl16_\w+)\s*\(", src)))


def test_header_symbols_are_exported():
    L = K.lib()
    names = declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(L, n), n
    assert set(names) <= set(K.EXPORTED) | set(names)


def test_strerror_covers_codes():
    for code in (0, -1, -2, -3, -4, -5, 1):
        assert K.irkgl16_strerror(code) != "unknown status"
    assert K.irkgl16_strerror(12345) == "unknown status"


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_create_without_gpu_reports_edevice():
    p = [dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)]
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create(p)
    assert e.value.code == K.IRKGL16_EDEVICE


@pytest.mark.parametrize("bad", [
    dict(kind=7, n=1, d=2),
    dict(kind=K.IRKGL16_KEPLER, n=2, d=2),
    dict(kind=K.IRKGL16_KEPLER, n=1, d=1),
    dict(kind=K.IRKGL16_GRAVITY, n=3, d=3),                       # no masses
    dict(kind=K.IRKGL16_GRAVITY, n=2, d=3, mass=[1.0, -1.0]),
    dict(kind=K.IRKGL16_GRAVITY, n=2, d=3, mass=[1.0, 1.0], eps=-1.0),
    dict(kind=K.IRKGL16_GRAVITY, n=2, d=3, mass=[1.0, np.nan]),
    dict(kind=K.IRKGL16_CHAIN, n=4, d=2),
    dict(kind=K.IRKGL16_CHAIN, n=4, d=1, beta=np.inf),
    dict(kind=K.IRKGL16_CHAIN, n=0, d=1),
])
def test_create_rejects_invalid_problems(bad):
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create([bad])
    assert e.value.code == K.IRKGL16_EINVAL


def test_null_arguments_rejected():
    L = K.lib()
    assert L.irkgl16_create(None, None, 0, None, None) == K.IRKGL16_EINVAL
    assert L.irkgl16_integrate(None, None, None, None, None, None, None, None, None) == K.IRKGL16_EINVAL
    assert L.irkgl16_last_stats(None, None) == K.IRKGL16_EINVAL
    L.irkgl16_destroy(None)  # NULL-safe


def test_product_table_matches_oracle_table(orc):
    """The library's coefficient header (its own generator) equals the oracle's
    table bit-for-bit."""
    src = open(os.path.join(ROOT, "paper_2511_03655_amd", "csrc", "irkgl16_coeffs.h")).read()

    def grab(name):
        m = re.search(name + r"\[8\](?:\[8\])? = \{(.*?)\};", src, re.S)
        return np.array([float.fromhex(x) for x in re.findall(r"-?0x[0-9a-fp.+-]+", m.group(1))])
    t = orc.tableau()
    for key, name in (("c", "kC"), ("b", "kB"), ("eta", "kEta"), ("mu", "kMu"), ("nu", "kNu")):
        assert np.array_equal(grab(name), t[key].ravel()), key


def test_folded_guess_matrix_matches_oracle_tableau():
    """The product's folded initial-guess matrix K = A W diag(1/b) (fused
    arithmetic mode) equals, entry by entry, the correctly rounded value of the
    same product formed from the oracle's independent high-precision tableau
    (eq. IRK_init2 with mu_sj b_j = a_sj and row sums of A equal to c)."""
    import mpmath
    from oracle import tableau as T
    src = open(os.path.join(ROOT, "paper_2511_03655_amd", "csrc", "irkgl16_coeffs.h")).read()
    m = re.search(r"kK\[8\]\[8\] = \{(.*?)\};", src, re.S)
    k = np.array([float.fromhex(x) for x in re.findall(r"-?0x[0-9a-fp.+-]+", m.group(1))])
    ex = T.exact_tableau()
    with mpmath.workdps(T.DPS):
        want = [T.rne(mpmath.fsum(ex["A"][s][j] * ex["W"][j][i] for j in range(8)) / ex["b"][i])
                for s in range(8) for i in range(8)]
        rows = [mpmath.fsum(ex["A"][s][j] for j in range(8)) - ex["c"][s] for s in range(8)]
    assert np.array_equal(k, np.array(want, dtype=np.float64))
    assert max(abs(float(r)) for r in rows) < 1e-90  # row sums of A are c


def test_graft_entry_build_compiles_everything(tmp_path):
    import importlib
    ge = importlib.import_module("__graft_entry__")
    ge.build()
    assert os.path.exists(os.path.join(ROOT, "paper_2511_03655_amd", "libirkgl16.so"))
    assert os.path.exists(os.path.join(ROOT, "oracle", "liborc.so"))


def test_user_force_compiles_without_gpu():
    from paper_2511_03655_amd import user_forces as UF
    rc, log = K.irkgl16_user_compile_check(UF.HENON_HEILES, 2)
    assert rc == K.IRKGL16_OK, log
    for src, dq in ((UF.HARMONIC, 6), (UF.HENON_HEILES_T, 2), (UF.DRIVEN, 3)):
        rc, log = K.irkgl16_user_compile_check(src, dq)
        assert rc == K.IRKGL16_OK, log


def test_user_force_compile_errors_are_reported():
    bad = "__device__ void irkgl16_user_force(const double* q, double* g, const double* prm,\n" \
          "                                   double t) {\n" \
          "  g[0] = -q[0]\n}\n"  # missing semicolon on line 3
    rc, log = K.irkgl16_user_compile_check(bad, 1)
    assert rc == K.IRKGL16_EINVAL
    assert "user_force:" in log and "error" in log
    rc, _ = K.irkgl16_user_compile_check("", 1)  # no force function defined
    assert rc == K.IRKGL16_EINVAL
    old = "__device__ void irkgl16_user_force(const double* q, double* g, const double* prm) {}"
    rc, _ = K.irkgl16_user_compile_check(old, 1)  # wrong signature (no time argument)
    assert rc == K.IRKGL16_EINVAL
    for dq in (0, 65, -3):
        rc, _ = K.irkgl16_user_compile_check("", dq)
        assert rc == K.IRKGL16_EINVAL
    L = K.lib()
    assert L.irkgl16_user_compile_check(None, 2, None, 0) == K.IRKGL16_EINVAL


def test_create_user_validates_arguments():
    from paper_2511_03655_amd import user_forces as UF
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create_user(UF.HARMONIC, 0, None, 4)
    assert e.value.code == K.IRKGL16_EINVAL
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create_user(UF.HARMONIC, 3, np.array([[1.0], [np.nan]]), 2)
    assert e.value.code == K.IRKGL16_EINVAL
    L = K.lib()
    assert L.irkgl16_create_user(None, None, 2, 0, None, 1, None, None) == K.IRKGL16_EINVAL


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_create_user_without_gpu_reports_edevice():
    from paper_2511_03655_amd import user_forces as UF
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create_user(UF.HENON_HEILES, 2, None, 3)
    assert e.value.code == K.IRKGL16_EDEVICE


def test_ode_sources_compile_without_gpu():
    from paper_2511_03655_amd import user_forces as UF
    for src, D in ((UF.OSC_RHS, 2), (UF.KEPLER_RHS, 6), (UF.DAMPED_RHS, 2), (UF.DRIVEN_RHS, 2),
                   (UF.SCHWARZSCHILD_RHS, 4), (UF.OSC_RHS, 16)):
        rc, log = K.irkgl16_ode_compile_check(src, D)
        assert rc == K.IRKGL16_OK, log
    # a second-order force is not a first-order right-hand side, and vice versa
    rc, _ = K.irkgl16_ode_compile_check(UF.HENON_HEILES, 2)
    assert rc == K.IRKGL16_EINVAL
    rc, _ = K.irkgl16_user_compile_check(UF.OSC_RHS, 2)
    assert rc == K.IRKGL16_EINVAL
    for D in (0, 65):
        rc, _ = K.irkgl16_ode_compile_check(UF.OSC_RHS, D)
        assert rc == K.IRKGL16_EINVAL


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_create_ode_without_gpu_reports_edevice():
    from paper_2511_03655_amd import user_forces as UF
    with pytest.raises(K.IRKGL16Error) as e:
        K.irkgl16_create_ode(UF.DAMPED_RHS, 2, np.array([[0.1]]), 1)
    assert e.value.code == K.IRKGL16_EDEVICE
    L = K.lib()
    assert L.irkgl16_create_ode(None, None, 2, 0, None, 1, None, None) == K.IRKGL16_EINVAL


def test_stage_count_validation():
    """s = 2, 4, 6 only for run-time compiled contexts; other counts rejected
    before any device work."""
    from paper_2511_03655_amd import user_forces as UF
    p = [dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)]
    L = K.lib()
    for st in (4, 3, 10, -1):
        arr = (K.irkgl16_problem * 1)()
        arr[0] = K.irkgl16_problem(0, 1, 2, None, None, 1.0, 0.0, 0.0)
        opt = K.irkgl16_options(0, 0, 0, st)
        ctx = C.c_void_p()
        assert L.irkgl16_create(C.byref(ctx), arr, 1, C.byref(opt), None) == K.IRKGL16_EINVAL, st
    for st in (3, 5, 10, 16):
        with pytest.raises(K.IRKGL16Error) as e:
            K.irkgl16_create_user(UF.HENON_HEILES, 2, None, 2, stages=st)
        assert e.value.code == K.IRKGL16_EINVAL
    del p


def test_product_tables_of_every_stage_count_match_oracle():
    """The library's flat tables for s = 2, 4, 6, 8 (its own generator) equal
    the oracle's independently generated binary64 tables entry for entry."""
    from oracle import tableau as T
    src = open(os.path.join(ROOT, "paper_2511_03655_amd", "csrc", "irkgl16_coeffs.h")).read()
    for s in (2, 4, 6, 8):
        m = re.search(rf"kTabS{s}\[(\d+)\] = \{{(.*?)\}};", src, re.S)
        flat = np.array([float.fromhex(x) for x in re.findall(r"-?0x[0-9a-fp.+-]+", m.group(2))])
        assert int(m.group(1)) == 2 * s + 4 * s * s == flat.size
        fp = T.fp64_tables(T.exact_tableau(s))
        want = np.concatenate([fp["c"], fp["b"], np.ravel(fp["eta"]), np.ravel(fp["mu"]),
                               np.ravel(fp["nu"])])
        assert np.array_equal(flat[:2 * s + 3 * s * s], want), s


def test_explicit_method_validation():
    """Explicit baselines only for second-order user contexts with s = 8;
    rejected before any device work."""
    from paper_2511_03655_amd import user_forces as UF
    L = K.lib()
    arr = (K.irkgl16_problem * 1)()
    arr[0] = K.irkgl16_problem(0, 1, 2, None, None, 1.0, 0.0, 0.0)
    ctx = C.c_void_p()
    opt = K.irkgl16_options(0, 0, 0, 0, K.IRKGL16_STRANG)
    assert L.irkgl16_create(C.byref(ctx), arr, 1, C.byref(opt), None) == K.IRKGL16_EINVAL
    for kw in (dict(method=3), dict(method=-1), dict(method=K.IRKGL16_SUZ90, stages=4)):
        with pytest.raises(K.IRKGL16Error) as e:
            K.irkgl16_create_user(UF.HENON_HEILES, 2, None, 2, **kw)
        assert e.value.code == K.IRKGL16_EINVAL, kw
    opt = K.irkgl16_options(0, 0, 0, 0, K.IRKGL16_SUZ90)
    assert L.irkgl16_create_ode(C.byref(ctx), UF.OSC_RHS.encode(), 2, 0, None, 1, C.byref(opt),
                                None) == K.IRKGL16_EINVAL


def test_product_splitting_tables_match_oracle():
    """The library's explicit-method tables (its own root finding for
    Suzuki's coefficient) equal the oracle's closed-form ones."""
    from oracle import tableau as T
    src = open(os.path.join(ROOT, "paper_2511_03655_amd", "csrc", "irkgl16_coeffs.h")).read()
    co = T.splitting_coefficients()
    for nm, key in (("Strang", "STRANG"), ("Suz90", "SUZ90")):
        m = re.search(rf"kSplit{nm}\[\d+\] = \{{(.*?)\}};", src, re.S)
        flat = [float.fromhex(x) for x in re.findall(r"-?0x[0-9a-fp.+-]+", m.group(1))]
        assert flat == co[key]["a"] + co[key]["b"] + co[key]["c"], nm


def test_one_hip_runtime_with_torch():
    """Loading the library in a fresh process and then importing torch leaves
    a single HIP runtime mapped (torch's bundled copy would otherwise come in
    beside the one this library links, and find no device)."""
    import subprocess
    import sys
    code = ("import re; from paper_2511_03655_amd import irkgl16 as K; K.lib(); import torch; "
            "m = open('/proc/self/maps').read(); "
            "print(sorted(set(re.findall(r'\\S*libamdhip64\\S*', m))))")
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                         cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                         timeout=300)
    assert out.returncode == 0, out.stderr
    import ast
    paths = ast.literal_eval(out.stdout.strip().splitlines()[-1])
    assert len(paths) == 1, paths


# ---- allocation-free entry point: argument and size checks come before any
# device call, so they hold without a GPU

def _static(problems, flags=0, h=0.1, nsteps=10, stride=10):
    return K.irkgl16_integrate_static(problems, 8, 8, h, nsteps, stride, 8, 8, flags=flags)


def test_static_entry_point_rejects_beyond_its_scratch():
    kep = dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)
    assert _static([kep] * (K.IRKGL16_STATIC_MAX_INST + 1)) == K.IRKGL16_ESCRATCH
    chain = dict(kind=K.IRKGL16_CHAIN, n=1024, d=1, beta=1.0)
    # 96 Dq bytes of state per chain: 400 chains of 1024 sites need 39 MB
    assert _static([chain] * 400) == K.IRKGL16_ESCRATCH


@pytest.mark.parametrize("case", ["plain", "graph", "large", "stride", "h"])
def test_static_entry_point_rejects_what_it_does_not_serve(case):
    kep = dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)
    if case == "plain":
        assert _static([kep], flags=K.IRKGL16_PLAIN) == K.IRKGL16_EINVAL
    elif case == "graph":
        assert _static([kep], flags=K.IRKGL16_PLAIN | K.IRKGL16_GRAPH) == K.IRKGL16_EINVAL
    elif case == "large":  # a system for the whole-GPU kernel
        big = dict(kind=K.IRKGL16_GRAVITY, n=600, d=3, mass=np.full(600, 1 / 600), G=1.0)
        assert _static([big]) == K.IRKGL16_EINVAL
    elif case == "stride":
        assert _static([kep], nsteps=10, stride=3) == K.IRKGL16_EINVAL
    else:
        assert _static([kep], h=float("nan")) == K.IRKGL16_EINVAL


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_static_entry_point_without_gpu_reports_edevice():
    kep = dict(kind=K.IRKGL16_KEPLER, n=1, d=2, G=1.0)
    assert _static([kep]) == K.IRKGL16_EDEVICE
    assert _static([]) == K.IRKGL16_OK  # nothing to do: no device needed


def test_serving_calls_reject_null_handles():
    """Without a server, every serving call reports EINVAL (no GPU needed)."""
    L = K.lib()
    info = K.irkgl16_server_info()
    assert L.irkgl16_cancel(None, 1) == K.IRKGL16_EINVAL
    assert L.irkgl16_server_stats(None, C.byref(info)) == K.IRKGL16_EINVAL
    assert K.irkgl16_strerror(K.IRKGL16_ECANCELED) == "the request was cancelled"

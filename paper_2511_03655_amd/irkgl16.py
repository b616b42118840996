"""ctypes binding of ``libirkgl16.so`` (C ABI in ``include/irkgl16.h``).

Argument marshalling only: every integration step runs in the library's HIP
kernels.  The functions carry the C names; :class:`Integrator` is a small
convenience wrapper around them.  Importing this module never falls back to
another implementation: if the library is missing or cannot be loaded,
:func:`lib` raises.

Host mode takes numpy arrays.  Device mode (``IRKGL16_DEVICE_PTRS``) takes
torch CUDA tensors (float64) whose memory the caller owns; the work is
enqueued on the stream given at creation and the caller synchronizes.
"""
from __future__ import annotations

import ctypes as C
import importlib.util
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# IRKGL16_LIB names another build of the same library (the CPU tests' sanitizer
# build); there is no other implementation to fall back to.
LIB_PATH = os.environ.get("IRKGL16_LIB") or os.path.join(HERE, "libirkgl16.so")

IRKGL16_OK, IRKGL16_EINVAL, IRKGL16_ENOMEM, IRKGL16_EDEVICE = 0, -1, -2, -3
IRKGL16_ENONFINITE, IRKGL16_ENOCONV, IRKGL16_ESCRATCH, IRKGL16_ECANCELED = -4, 1, -5, -6
IRKGL16_STATIC_SCRATCH_BYTES, IRKGL16_STATIC_MAX_INST = 32 << 20, 16384
IRKGL16_KEPLER, IRKGL16_GRAVITY, IRKGL16_CHAIN = 0, 1, 2
IRKGL16_DEVICE_PTRS, IRKGL16_PLAIN, IRKGL16_REPRODUCIBLE, IRKGL16_GRAPH = 1, 2, 4, 8
IRKGL16_STRANG, IRKGL16_SUZ90 = 1, 2  # irkgl16_options.method: explicit baselines

EXPORTED = ["irkgl16_create", "irkgl16_integrate", "irkgl16_last_stats", "irkgl16_destroy",
            "irkgl16_strerror", "irkgl16_server_create", "irkgl16_submit", "irkgl16_poll",
            "irkgl16_wait", "irkgl16_server_destroy", "irkgl16_create_user",
            "irkgl16_user_compile_check", "irkgl16_create_ode", "irkgl16_ode_compile_check",
            "irkgl16_integrate_static", "irkgl16_cancel", "irkgl16_server_stats"]


class irkgl16_problem(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n", C.c_int32), ("d", C.c_int32),
                ("mass", C.POINTER(C.c_double)), ("coupling", C.POINTER(C.c_double)),
                ("G", C.c_double), ("eps", C.c_double), ("beta", C.c_double)]


class irkgl16_options(C.Structure):
    _fields_ = [("max_iter", C.c_int32), ("record_iters", C.c_int32), ("flags", C.c_uint32),
                ("stages", C.c_int32), ("method", C.c_int32)]


class irkgl16_stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("iterations", C.c_int64),
                ("nonconverged_steps", C.c_int64), ("max_k", C.c_int32),
                ("n_nonfinite", C.c_int32), ("device_ms", C.c_double),
                ("inst_iterations", C.POINTER(C.c_int64)), ("inst_status", C.POINTER(C.c_int32)),
                ("step_iters", C.POINTER(C.c_uint8))]


class irkgl16_server_options(C.Structure):
    _fields_ = [("cap_bytes", C.c_int64), ("slice_steps", C.c_int64), ("max_iter", C.c_int32),
                ("max_resident", C.c_int32), ("flags", C.c_uint32), ("slice_ms", C.c_double)]


class irkgl16_request_info(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps", C.c_int64), ("iterations", C.c_int64),
                ("submit_s", C.c_double), ("admit_s", C.c_double), ("done_s", C.c_double)]


class irkgl16_server_info(C.Structure):
    _fields_ = [("slices", C.c_int64), ("slice_wall_s", C.c_double), ("slice_device_s", C.c_double),
                ("requests_done", C.c_int64), ("requests_cancelled", C.c_int64),
                ("max_resident", C.c_int32), ("resident", C.c_int32), ("pending", C.c_int32)]


class IRKGL16Error(RuntimeError):
    def __init__(self, code, what=""):
        self.code = code
        super().__init__(f"{what}: {irkgl16_strerror(code)} ({code})")


_lib = None


def lib():
    """Load the HIP library (raises if it is not built or cannot be loaded)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2511_03655_amd/build.py")
        # torch ships its own HIP runtime and asks for it under a name that a
        # runtime loaded for this library does not answer to: loading this
        # library first leaves two HIP runtimes in the process, and the second
        # (torch's) finds no device.  Loaded after torch, this library binds to
        # torch's copy, so one runtime serves both.
        if "torch" not in sys.modules and importlib.util.find_spec("torch") is not None:
            import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        dp, i64p = C.POINTER(C.c_double), C.POINTER(C.c_int64)
        L.irkgl16_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(irkgl16_problem), C.c_int32,
                                     C.POINTER(irkgl16_options), C.c_void_p]
        L.irkgl16_create.restype = C.c_int
        L.irkgl16_integrate.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, dp, i64p, i64p,
                                        C.c_void_p, C.c_void_p, C.POINTER(irkgl16_stats)]
        L.irkgl16_integrate.restype = C.c_int
        L.irkgl16_last_stats.argtypes = [C.c_void_p, C.POINTER(irkgl16_stats)]
        L.irkgl16_last_stats.restype = C.c_int
        L.irkgl16_destroy.argtypes = [C.c_void_p]
        L.irkgl16_destroy.restype = None
        L.irkgl16_strerror.argtypes = [C.c_int]
        L.irkgl16_strerror.restype = C.c_char_p
        L.irkgl16_server_create.argtypes = [C.POINTER(C.c_void_p),
                                            C.POINTER(irkgl16_server_options), C.c_void_p]
        L.irkgl16_server_create.restype = C.c_int
        L.irkgl16_submit.argtypes = [C.c_void_p, C.POINTER(irkgl16_problem), dp, dp, C.c_double,
                                     C.c_int64, C.c_int64, C.POINTER(C.c_int64)]
        L.irkgl16_submit.restype = C.c_int
        L.irkgl16_poll.argtypes = [C.c_void_p, C.c_int64, C.POINTER(C.c_int32)]
        L.irkgl16_poll.restype = C.c_int
        L.irkgl16_wait.argtypes = [C.c_void_p, C.c_int64, dp, dp, C.POINTER(irkgl16_request_info)]
        L.irkgl16_wait.restype = C.c_int
        L.irkgl16_cancel.argtypes = [C.c_void_p, C.c_int64]
        L.irkgl16_cancel.restype = C.c_int
        L.irkgl16_server_stats.argtypes = [C.c_void_p, C.POINTER(irkgl16_server_info)]
        L.irkgl16_server_stats.restype = C.c_int
        L.irkgl16_server_destroy.argtypes = [C.c_void_p]
        L.irkgl16_server_destroy.restype = None
        L.irkgl16_create_user.argtypes = [C.POINTER(C.c_void_p), C.c_char_p, C.c_int32, C.c_int32,
                                          dp, C.c_int32, C.POINTER(irkgl16_options), C.c_void_p]
        L.irkgl16_create_user.restype = C.c_int
        L.irkgl16_user_compile_check.argtypes = [C.c_char_p, C.c_int32, C.c_char_p, C.c_int64]
        L.irkgl16_user_compile_check.restype = C.c_int
        L.irkgl16_create_ode.argtypes = L.irkgl16_create_user.argtypes
        L.irkgl16_create_ode.restype = C.c_int
        L.irkgl16_ode_compile_check.argtypes = [C.c_char_p, C.c_int32, C.c_char_p, C.c_int64]
        L.irkgl16_ode_compile_check.restype = C.c_int
        L.irkgl16_integrate_static.argtypes = [C.POINTER(irkgl16_problem), C.c_int32,
                                               C.POINTER(irkgl16_options), C.c_void_p,
                                               C.c_void_p, C.c_void_p, dp, i64p, i64p,
                                               C.c_void_p, C.c_void_p, C.POINTER(irkgl16_stats)]
        L.irkgl16_integrate_static.restype = C.c_int
        _lib = L
    return _lib


def irkgl16_strerror(code):
    return lib().irkgl16_strerror(int(code)).decode()


def _ptr(x):
    """Address of a numpy array or a torch tensor (no copies)."""
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return C.c_void_p(x.data_ptr())
    return C.c_void_p(x.ctypes.data)


def irkgl16_create(problems, max_iter=0, record_iters=False, flags=0, stream=None):
    """problems: list of dicts with kind, n, d, mass, coupling, G, eps, beta.

    Returns (ctx_handle, keepalive).  stream: a hipStream_t address or a torch
    stream (its raw handle is passed).
    """
    n = len(problems)
    arr = (irkgl16_problem * max(n, 1))()
    keep = []
    for i, p in enumerate(problems):
        mass = p.get("mass")
        coup = p.get("coupling")
        m = None if mass is None else np.ascontiguousarray(mass, np.float64)
        c = None if coup is None else np.ascontiguousarray(coup, np.float64)
        keep += [m, c]
        arr[i] = irkgl16_problem(int(p["kind"]), int(p["n"]), int(p["d"]),
                                 m.ctypes.data_as(C.POINTER(C.c_double)) if m is not None else None,
                                 c.ctypes.data_as(C.POINTER(C.c_double)) if c is not None else None,
                                 float(p.get("G", 1.0)), float(p.get("eps", 0.0)),
                                 float(p.get("beta", 0.0)))
    opt = irkgl16_options(int(max_iter), int(bool(record_iters)), int(flags))
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    ctx = C.c_void_p()
    rc = lib().irkgl16_create(C.byref(ctx), arr, n, C.byref(opt),
                              C.c_void_p(stream) if stream else None)
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_create")
    return ctx


def irkgl16_create_user(force_src, dq, params, n_inst, max_iter=0, record_iters=False, flags=0,
                        stream=None, stages=0, method=0):
    """Context for n_inst instances of a force given as device source.

    params: array of shape (n_inst, n_params) (or None for no parameters).
    """
    prm = None if params is None else np.ascontiguousarray(params, np.float64).reshape(n_inst, -1)
    n_params = 0 if prm is None else prm.shape[1]
    opt = irkgl16_options(int(max_iter), int(bool(record_iters)), int(flags), int(stages),
                          int(method))
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    ctx = C.c_void_p()
    rc = lib().irkgl16_create_user(
        C.byref(ctx), force_src.encode(), int(dq), int(n_params),
        prm.ctypes.data_as(C.POINTER(C.c_double)) if n_params > 0 else None, int(n_inst),
        C.byref(opt), C.c_void_p(stream) if stream else None)
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_create_user")
    return ctx


def irkgl16_user_compile_check(force_src, dq, log_len=1 << 16):
    """Returns (status, compiler log)."""
    buf = C.create_string_buffer(log_len)
    rc = lib().irkgl16_user_compile_check(force_src.encode(), int(dq), buf, log_len)
    return rc, buf.value.decode(errors="replace")


def irkgl16_create_ode(rhs_src, D, params, n_inst, max_iter=0, record_iters=False, flags=0,
                       stream=None, stages=0):
    """First-order context (y' = f(t, y)) for n_inst instances of D components."""
    prm = None if params is None else np.ascontiguousarray(params, np.float64).reshape(n_inst, -1)
    n_params = 0 if prm is None else prm.shape[1]
    opt = irkgl16_options(int(max_iter), int(bool(record_iters)), int(flags), int(stages))
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    ctx = C.c_void_p()
    rc = lib().irkgl16_create_ode(
        C.byref(ctx), rhs_src.encode(), int(D), int(n_params),
        prm.ctypes.data_as(C.POINTER(C.c_double)) if n_params > 0 else None, int(n_inst),
        C.byref(opt), C.c_void_p(stream) if stream else None)
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_create_ode")
    return ctx


def irkgl16_ode_compile_check(rhs_src, D, log_len=1 << 16):
    """Returns (status, compiler log)."""
    buf = C.create_string_buffer(log_len)
    rc = lib().irkgl16_ode_compile_check(rhs_src.encode(), int(D), buf, log_len)
    return rc, buf.value.decode(errors="replace")


def irkgl16_integrate(ctx, q0, p0, h, nsteps, out_stride, q_out, p_out, stats=None):
    h = np.ascontiguousarray(h, np.float64)
    ns = np.ascontiguousarray(nsteps, np.int64)
    sd = np.ascontiguousarray(out_stride, np.int64)
    return lib().irkgl16_integrate(ctx, _ptr(q0), _ptr(p0),
                                   h.ctypes.data_as(C.POINTER(C.c_double)),
                                   ns.ctypes.data_as(C.POINTER(C.c_int64)),
                                   sd.ctypes.data_as(C.POINTER(C.c_int64)), _ptr(q_out),
                                   _ptr(p_out), C.byref(stats) if stats is not None else None)


def irkgl16_integrate_static(problems, q0, p0, h, nsteps, out_stride, q_out, p_out,
                             max_iter=0, record_iters=False, flags=0, stream=None, stats=None):
    """Allocation-free integration (create + integrate + destroy in one call,
    scratch in the library's fixed device array).  q0, p0, q_out, p_out: torch
    CUDA tensors (float64) or raw device addresses; h, nsteps, out_stride: one
    value per instance (host).  stats: an irkgl16_stats or None.  Returns the
    status code."""
    keep = []
    n = len(problems)
    arr = (irkgl16_problem * max(n, 1))()
    for i, p in enumerate(problems):
        arr[i] = _problem_struct(p, keep)
    opt = irkgl16_options(int(max_iter), int(bool(record_iters)), int(flags))
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    h = np.ascontiguousarray(np.broadcast_to(np.asarray(h, np.float64), (n,)))
    ns = np.ascontiguousarray(np.broadcast_to(np.asarray(nsteps, np.int64), (n,)))
    sd = np.ascontiguousarray(np.broadcast_to(np.asarray(out_stride, np.int64), (n,)))

    def addr(x):
        return C.c_void_p(int(x)) if isinstance(x, int) else _ptr(x)

    return lib().irkgl16_integrate_static(
        arr, n, C.byref(opt), C.c_void_p(stream) if stream else None, addr(q0), addr(p0),
        h.ctypes.data_as(C.POINTER(C.c_double)), ns.ctypes.data_as(C.POINTER(C.c_int64)),
        sd.ctypes.data_as(C.POINTER(C.c_int64)), addr(q_out), addr(p_out),
        C.byref(stats) if stats is not None else None)


def irkgl16_last_stats(ctx, stats):
    return lib().irkgl16_last_stats(ctx, C.byref(stats))


def irkgl16_destroy(ctx):
    if ctx:
        lib().irkgl16_destroy(ctx)


class Integrator:
    """Owns one context.  Packing follows the C ABI: instances concatenated."""

    def __init__(self, problems, max_iter=0, record_iters=False, flags=0, stream=None):
        self.problems = list(problems)
        self.dq = np.array([int(p["n"]) * int(p["d"]) for p in self.problems], np.int64)
        self.flags = int(flags)
        self.record_iters = bool(record_iters)
        self.ctx = irkgl16_create(self.problems, max_iter, record_iters, flags, stream)

    @classmethod
    def user(cls, force_src, dq, n_inst, params=None, max_iter=0, record_iters=False, flags=0,
             stream=None, stages=0, method=0):
        """Integrator of n_inst instances of a user force (irkgl16_create_user)."""
        self = cls.__new__(cls)
        self.problems = [dict(kind=-1, n=1, d=int(dq))] * int(n_inst)
        self.dq = np.full(int(n_inst), int(dq), np.int64)
        self.flags = int(flags)
        self.record_iters = bool(record_iters)
        self.ctx = None
        self.ctx = irkgl16_create_user(force_src, dq, params, n_inst, max_iter, record_iters,
                                       flags, stream, stages, method)
        return self

    @classmethod
    def ode(cls, rhs_src, D, n_inst, params=None, max_iter=0, record_iters=False, flags=0,
            stream=None, stages=0):
        """Integrator of n_inst first-order instances (irkgl16_create_ode): y0 is
        passed as q0; integrate returns the y frames as q_out (p_out is None)."""
        self = cls.__new__(cls)
        self.problems = [dict(kind=-2, n=1, d=int(D))] * int(n_inst)
        self.dq = np.full(int(n_inst), int(D), np.int64)
        self.flags = int(flags)
        self.record_iters = bool(record_iters)
        self.is_ode = True
        self.ctx = None
        self.ctx = irkgl16_create_ode(rhs_src, D, params, n_inst, max_iter, record_iters, flags,
                                      stream, stages)
        return self

    def close(self):
        """Release the context (synchronizes its stream, frees its device memory)."""
        ctx = getattr(self, "ctx", None)
        if ctx and _lib is not None:
            self.ctx = None
            _lib.irkgl16_destroy(ctx)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        # During interpreter shutdown the HIP runtime, a caller-owned stream or
        # an attached profiler may already be gone: destroying the context then
        # (a stream synchronization and hipFree) is not safe, and the process is
        # about to release the device anyway.  Close contexts explicitly.
        if not sys.is_finalizing():
            self.close()

    def frames(self, nsteps, stride):
        return np.asarray(nsteps, np.int64) // np.asarray(stride, np.int64) + 1

    def integrate(self, q0, p0, h, nsteps, out_stride, q_out=None, p_out=None, check=True):
        """Host mode: numpy in, numpy out.  Returns (q_out, p_out, stats dict, rc)."""
        n = len(self.problems)
        h = np.broadcast_to(np.asarray(h, np.float64), (n,))
        ns = np.broadcast_to(np.asarray(nsteps, np.int64), (n,))
        sd = np.broadcast_to(np.asarray(out_stride, np.int64), (n,))
        total = int(np.sum(self.dq * (ns // np.maximum(sd, 1) + 1)))
        dev = bool(self.flags & IRKGL16_DEVICE_PTRS)
        ode = getattr(self, "is_ode", False)
        if not dev:
            q0 = np.ascontiguousarray(q0, np.float64)
            p0 = None if ode else np.ascontiguousarray(p0, np.float64)
            if q_out is None:
                q_out = np.empty(total)
            if p_out is None and not ode:
                p_out = np.empty(total)
        st = irkgl16_stats()
        inst_it = np.zeros(n, np.int64)
        inst_st = np.zeros(n, np.int32)
        st.inst_iterations = inst_it.ctypes.data_as(C.POINTER(C.c_int64))
        st.inst_status = inst_st.ctypes.data_as(C.POINTER(C.c_int32))
        step_it = None
        if self.record_iters:
            step_it = np.zeros(int(np.sum(ns)), np.uint8)
            st.step_iters = step_it.ctypes.data_as(C.POINTER(C.c_uint8))
        rc = irkgl16_integrate(self.ctx, q0, p0, h, ns, sd, q_out, p_out,
                               None if dev else st)
        if check and rc < 0 and rc != IRKGL16_ENONFINITE:
            raise IRKGL16Error(rc, "irkgl16_integrate")
        if dev:
            return q_out, p_out, None, rc
        return q_out, p_out, dict(steps=st.steps, iterations=st.iterations,
                                  nonconverged_steps=st.nonconverged_steps, max_k=st.max_k,
                                  n_nonfinite=st.n_nonfinite, device_ms=st.device_ms,
                                  inst_iterations=inst_it, inst_status=inst_st,
                                  step_iters=step_it), rc

    def last_stats(self):
        n = len(self.problems)
        st = irkgl16_stats()
        inst_it = np.zeros(n, np.int64)
        inst_st = np.zeros(n, np.int32)
        st.inst_iterations = inst_it.ctypes.data_as(C.POINTER(C.c_int64))
        st.inst_status = inst_st.ctypes.data_as(C.POINTER(C.c_int32))
        rc = irkgl16_last_stats(self.ctx, st)
        return dict(steps=st.steps, iterations=st.iterations,
                    nonconverged_steps=st.nonconverged_steps, max_k=st.max_k,
                    n_nonfinite=st.n_nonfinite, device_ms=st.device_ms,
                    inst_iterations=inst_it, inst_status=inst_st), rc


def split_frames(flat, dq, nframes):
    """Unpack a packed output array into a list of (frames, Dq) arrays."""
    out, off = [], 0
    for d, f in zip(np.atleast_1d(dq), np.atleast_1d(nframes)):
        out.append(np.asarray(flat[off:off + d * f]).reshape(f, d))
        off += d * f
    return out


# ---------------------------------------------------------------- serving

def _problem_struct(p, keep):
    mass, coup = p.get("mass"), p.get("coupling")
    m = None if mass is None else np.ascontiguousarray(mass, np.float64)
    c = None if coup is None else np.ascontiguousarray(coup, np.float64)
    keep += [m, c]
    return irkgl16_problem(int(p["kind"]), int(p["n"]), int(p["d"]),
                           m.ctypes.data_as(C.POINTER(C.c_double)) if m is not None else None,
                           c.ctypes.data_as(C.POINTER(C.c_double)) if c is not None else None,
                           float(p.get("G", 1.0)), float(p.get("eps", 0.0)),
                           float(p.get("beta", 0.0)))


def irkgl16_server_create(cap_bytes, slice_steps=0, max_iter=0, max_resident=0, flags=0,
                          stream=None, slice_ms=0.0):
    opt = irkgl16_server_options(int(cap_bytes), int(slice_steps), int(max_iter),
                                 int(max_resident), int(flags), float(slice_ms))
    if stream is not None and hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    srv = C.c_void_p()
    rc = lib().irkgl16_server_create(C.byref(srv), C.byref(opt),
                                     C.c_void_p(stream) if stream else None)
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_server_create")
    return srv


def irkgl16_submit(srv, problem, q0, p0, h, nsteps, out_stride):
    keep = []
    pr = _problem_struct(problem, keep)
    q0 = np.ascontiguousarray(q0, np.float64)
    p0 = np.ascontiguousarray(p0, np.float64)
    t = C.c_int64()
    rc = lib().irkgl16_submit(srv, C.byref(pr), q0.ctypes.data_as(C.POINTER(C.c_double)),
                              p0.ctypes.data_as(C.POINTER(C.c_double)), float(h), int(nsteps),
                              int(out_stride), C.byref(t))
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_submit")
    return t.value


def irkgl16_poll(srv, ticket):
    done = C.c_int32()
    rc = lib().irkgl16_poll(srv, int(ticket), C.byref(done))
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_poll")
    return bool(done.value)


def irkgl16_wait(srv, ticket, q_out=None, p_out=None):
    info = irkgl16_request_info()
    dp = C.POINTER(C.c_double)
    rc = lib().irkgl16_wait(srv, int(ticket),
                            q_out.ctypes.data_as(dp) if q_out is not None else None,
                            p_out.ctypes.data_as(dp) if p_out is not None else None,
                            C.byref(info))
    return rc, dict(status=info.status, steps=info.steps, iterations=info.iterations,
                    submit_s=info.submit_s, admit_s=info.admit_s, done_s=info.done_s)


def irkgl16_cancel(srv, ticket):
    rc = lib().irkgl16_cancel(srv, int(ticket))
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_cancel")


def irkgl16_server_stats(srv):
    info = irkgl16_server_info()
    rc = lib().irkgl16_server_stats(srv, C.byref(info))
    if rc != IRKGL16_OK:
        raise IRKGL16Error(rc, "irkgl16_server_stats")
    return {k: getattr(info, k) for k, _ in irkgl16_server_info._fields_}


def irkgl16_server_destroy(srv):
    if srv:
        lib().irkgl16_server_destroy(srv)


class Server:
    """Owns one serving thread (continuous batching)."""

    def __init__(self, cap_bytes=1 << 30, slice_steps=1000, max_iter=0, max_resident=0, flags=0,
                 stream=None, slice_ms=0.0):
        self.srv = irkgl16_server_create(cap_bytes, slice_steps, max_iter, max_resident, flags,
                                         stream, slice_ms)
        self._dq = {}

    def submit(self, problem, q0, p0, h, nsteps, out_stride):
        t = irkgl16_submit(self.srv, problem, q0, p0, h, nsteps, out_stride)
        self._dq[t] = (int(problem["n"]) * int(problem["d"]), int(nsteps) // int(out_stride) + 1)
        return t

    def poll(self, ticket):
        return irkgl16_poll(self.srv, ticket)

    def wait(self, ticket, keep_frames=True):
        dq, nf = self._dq.pop(ticket)
        q = np.empty(dq * nf) if keep_frames else None
        p = np.empty(dq * nf) if keep_frames else None
        rc, info = irkgl16_wait(self.srv, ticket, q, p)
        return q, p, info, rc

    def cancel(self, ticket):
        irkgl16_cancel(self.srv, ticket)

    def stats(self):
        return irkgl16_server_stats(self.srv)

    def close(self):
        """Stop the serving thread after the pending requests and release the server."""
        if getattr(self, "srv", None):
            irkgl16_server_destroy(self.srv)
            self.srv = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        if not sys.is_finalizing():  # as Integrator.__del__
            self.close()


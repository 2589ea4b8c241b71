"""Python binding of libw1 (include/w1.h): argument marshalling only.

Every step of the solver runs in the HIP library; this module converts
arguments (NumPy arrays for host buffers, torch tensors on the GPU for
device buffers) into the C ABI's plain pointers and sizes.  It fails loudly
when the library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("W1_LIB_PATH") or os.path.join(HERE, "libw1.so")

W1_OK, W1_EAGAIN = 0, 1
W1_EINVAL, W1_ENOMEM, W1_EBUSY, W1_EDEVICE, W1_ESTATE, W1_ENOTFOUND = -1, -2, -3, -4, -5, -6
SOLVE_OK, SOLVE_MAXITER, SOLVE_DIVERGED, SOLVE_REJECTED, SOLVE_FAILED = 0, 1, 2, 3, 4
METRIC_L1, METRIC_L2, METRIC_LINF = 1, 2, 3
ALGO_PLAIN, ALGO_PROX = 1, 2
FP32, FP64 = 1, 2
STOP_KKT, STOP_FPR = 1, 2
FLAG_NO_RESIDENT, FLAG_NO_CERT, FLAG_LEVEL_COST, FLAG_NO_FIELDS = 1, 2, 4, 8
MAX_LEVELS = 12
FAM_PLAIN_TILED, FAM_PLAIN_RESIDENT, FAM_DCT, FAM_PROX_ELEM, FAM_OTHER = 0, 1, 2, 3, 4
FAMILIES = {0: "plain_tiled", 1: "plain_resident", 2: "dct", 3: "prox_elem", 4: "other", 5: "prox_resident"}


class W1Error(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} ({status})")


class Params(C.Structure):
    _fields_ = [
        ("n", C.c_int32), ("levels", C.c_int32), ("metric", C.c_int32), ("algo", C.c_int32),
        ("precision", C.c_int32), ("stop_rule", C.c_int32), ("tol", C.c_double), ("alpha", C.c_double),
        ("step_scale", C.c_double), ("max_iters", C.c_int32), ("check_every", C.c_int32),
        ("block_steps", C.c_int32), ("flags", C.c_int32), ("h", C.c_double),
        ("level_caps", C.c_int32 * MAX_LEVELS), ("diverge_window", C.c_int32), ("reserved", C.c_int32),
    ]


class Result(C.Structure):
    _fields_ = [
        ("w1", C.c_double), ("dual", C.c_double), ("lo", C.c_double), ("hi", C.c_double), ("kkt", C.c_double),
        ("status", C.c_int32), ("levels_run", C.c_int32), ("iters", C.c_int32 * MAX_LEVELS),
        ("measure", C.c_double * MAX_LEVELS), ("seconds", C.c_double), ("queue_seconds", C.c_double),
        ("level_w1", C.c_double * MAX_LEVELS), ("level_seconds", C.c_double * MAX_LEVELS),
    ]

    def as_dict(self):
        L = self.levels_run
        return {"w1": self.w1, "dual": self.dual, "lo": self.lo, "hi": self.hi, "kkt": self.kkt,
                "status": self.status, "levels_run": L, "iters": list(self.iters[:L]),
                "measure": list(self.measure[:L]), "seconds": self.seconds,
                "queue_seconds": self.queue_seconds, "level_w1": list(self.level_w1[:L]),
                "level_seconds": list(self.level_seconds[:L])}


_lib = None


def lib():
    """Load libw1.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1810_00118_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, dp = C.c_void_p, C.c_int32, C.POINTER(C.c_double)
    sig = {
        "w1_params_default": (None, [C.POINTER(Params)]),
        "w1_params_check": (C.c_int, [C.POINTER(Params)]),
        "w1_bytes_per_solve": (C.c_size_t, [C.POINTER(Params)]),
        "w1_plan": (C.c_int, [C.POINTER(Params), i32, C.c_size_t, vp, C.POINTER(vp)]),
        "w1_solve": (C.c_int, [vp, i32, C.POINTER(vp), C.POINTER(vp), i32, C.POINTER(Result)]),
        "w1_fields": (C.c_int, [vp, i32, vp, vp, vp, i32]),
        "w1_serve_config": (C.c_int, [vp, i32]),
        "w1_submit": (C.c_int, [vp, C.POINTER(Params), vp, vp, i32, C.POINTER(C.c_uint64)]),
        "w1_poll": (C.c_int, [vp, C.c_uint64, C.POINTER(Result), vp, vp, vp]),
        "w1_drain": (C.c_int, [vp]),
        "w1_serve_stats": (C.c_int, [vp, C.POINTER(C.c_int64)]),
        "w1_engine_counters": (C.c_int, [vp, C.POINTER(C.c_int64)]),
        "w1_destroy": (C.c_int, [vp]),
        "w1_trim_cache": (C.c_int, [C.POINTER(C.c_size_t)]),
        "w1_strerror": (C.c_char_p, [C.c_int]),
        "w1_version": (C.c_char_p, []),
        "w1_profile": (C.c_int, [vp, i32]),
        "w1_kernel_stats": (C.c_int, [vp, i32, dp]),
        "w1_tuner_table": (C.c_int, [C.c_char_p, C.c_size_t]),
        "w1_tuner_reset": (C.c_int, []),
        "w1_op_prepare": (C.c_int, [i32, i32, i32, vp, vp, C.POINTER(vp), vp]),
        "w1_op_prolong": (C.c_int, [i32, i32, vp, vp, vp, vp, vp, vp, vp]),
        "w1_op_plain_steps": (C.c_int, [i32, i32, i32, C.c_double, i32, i32, i32, i32, i32, vp, vp, vp, vp, dp,
                                        vp]),
        "w1_op_prox_steps": (C.c_int, [i32, i32, i32, C.c_double, i32, i32, vp, vp, vp, vp, vp, vp, vp, dp, vp]),
        "w1_op_poisson": (C.c_int, [i32, i32, vp, vp, vp]),
        "w1_op_poisson_noalloc": (C.c_int, [i32, i32, vp, vp, vp]),
        "w1_noalloc_bytes": (C.c_size_t, []),
        "w1_op_potential": (C.c_int, [i32, i32, vp, vp, vp, vp]),
        "w1_op_evaluate": (C.c_int, [i32, i32, i32, vp, vp, vp, vp, dp, vp]),
        "w1_solve3d": (C.c_int, [C.POINTER(Params), vp, vp, i32, C.POINTER(Result), vp, vp, vp]),
        "w1_solve3d_batch": (C.c_int, [C.POINTER(Params), i32, C.POINTER(vp), C.POINTER(vp), i32,
                                       C.POINTER(Result), i32]),
        "w1_op_plain_steps3d": (C.c_int, [i32, i32, i32, C.c_double, i32, vp, vp, vp, vp, vp, dp, vp]),
        "w1_op_prox_steps3d": (C.c_int, [i32, i32, i32, C.c_double, i32] + [vp] * 10 + [dp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def strerror(status):
    try:
        return lib().w1_strerror(int(status)).decode()
    except ImportError:
        return str(status)


def version():
    return lib().w1_version().decode()


def _check(st, what):
    if st != W1_OK:
        raise W1Error(st, what)


def params(**kw) -> Params:
    p = Params()
    lib().w1_params_default(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        if k == "level_caps":
            caps = list(v) + [0] * (MAX_LEVELS - len(v))
            v = (C.c_int32 * MAX_LEVELS)(*caps)
        setattr(p, k, v)
    return p


def bytes_per_solve(p: Params) -> int:
    return int(lib().w1_bytes_per_solve(C.byref(p)))


def check_params(p: Params) -> int:
    return int(lib().w1_params_check(C.byref(p)))


# ---------------------------------------------------------------------------
# buffers
# ---------------------------------------------------------------------------
def _ptr(x, dtype=None, on_device=None):
    """(pointer, is_device) of a contiguous NumPy array or torch tensor."""
    if x is None:
        return None, None
    mod = type(x).__module__
    if mod.startswith("torch"):
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        if dtype is not None and str(x.dtype).replace("torch.", "") != dtype:
            raise TypeError(f"expected {dtype}, got {x.dtype}")
        return C.c_void_p(x.data_ptr()), bool(x.is_cuda)
    a = x
    if not isinstance(a, np.ndarray) or not a.flags.c_contiguous:
        raise TypeError("expected a C-contiguous numpy array or torch tensor")
    if dtype is not None and a.dtype != np.dtype(dtype):
        raise TypeError(f"expected {dtype}, got {a.dtype}")
    return C.c_void_p(a.ctypes.data), False


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    return C.c_void_p(int(stream))


# ---------------------------------------------------------------------------
# solver handle
# ---------------------------------------------------------------------------
class Solver:
    """A w1_plan handle: batched solves (solve) and served mode (submit/poll)."""

    def __init__(self, p: Params, capacity: int = 1, hbm_budget: int = 0, stream=None):
        self.p = p
        self.capacity = capacity
        h = C.c_void_p()
        _check(lib().w1_plan(C.byref(p), capacity, hbm_budget, stream and C.c_void_p(int(stream)), C.byref(h)),
               "w1_plan")
        self.h = h
        self._keep = []

    def close(self):
        if self.h:
            lib().w1_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def solve(self, pairs):
        """pairs: list of (p0, p1) float64 arrays (host) or cuda tensors."""
        k = len(pairs)
        A = (C.c_void_p * k)()
        B = (C.c_void_p * k)()
        dev = None
        for i, (a, b) in enumerate(pairs):
            pa, da = _ptr(a, "float64")
            pb, db = _ptr(b, "float64")
            if dev is None:
                dev = da
            if da != dev or db != dev:
                raise ValueError("all masses must be on the same side (host or device)")
            A[i], B[i] = pa, pb
        out = (Result * k)()
        _check(lib().w1_solve(self.h, k, A, B, 1 if dev else 0, out), "w1_solve")
        return [r.as_dict() for r in out]

    def fields(self, index: int):
        """Finest-level (m1, m2, psi) of pair `index` of the last solve (host float64)."""
        n = self.p.n
        m1 = np.empty((n + 1, n + 1))
        m2 = np.empty_like(m1)
        psi = np.empty_like(m1)
        _check(lib().w1_fields(self.h, index, m1.ctypes.data, m2.ctypes.data, psi.ctypes.data, 0), "w1_fields")
        return m1, m2, psi

    def serve_config(self, queue_limit: int):
        _check(lib().w1_serve_config(self.h, queue_limit), "w1_serve_config")

    def submit(self, p0, p1, p: Params = None) -> int:
        pa, da = _ptr(p0, "float64")
        pb, db = _ptr(p1, "float64")
        t = C.c_uint64()
        _check(lib().w1_submit(self.h, C.byref(p) if p is not None else None, pa, pb, 1 if da else 0,
                               C.byref(t)), "w1_submit")
        return int(t.value)

    def poll(self, ticket: int, n: int = None, fields: bool = False):
        """None while running; else (result dict, fields or None)."""
        r = Result()
        bufs = [None, None, None]
        if fields:
            bufs = [np.empty((n + 1, n + 1)) for _ in range(3)]
        st = lib().w1_poll(self.h, ticket, C.byref(r), *[b.ctypes.data if b is not None else None for b in bufs])
        if st == W1_EAGAIN:
            return None
        _check(st, "w1_poll")
        return r.as_dict(), (tuple(bufs) if fields else None)

    def profile(self, enable=True, every=1):
        """Per-launch kernel timing on (every >= 1: about one launch in `every`) or off."""
        _check(lib().w1_profile(self.h, int(every) if enable else 0), "w1_profile")

    def kernel_stats(self):
        out = {}
        for f, name in FAMILIES.items():
            o = (C.c_double * 6)()
            _check(lib().w1_kernel_stats(self.h, f, o), "w1_kernel_stats")
            out[name] = {"launches": int(o[0]), "ms": o[1], "node_updates": o[2], "alg_bytes": o[3],
                         "flops": o[4], "issued": int(o[5])}
        return out

    def drain(self):
        _check(lib().w1_drain(self.h), "w1_drain")

    def counters(self):
        o = (C.c_int64 * 5)()
        _check(lib().w1_engine_counters(self.h, o), "w1_engine_counters")
        return {"host_steps": o[0], "level_starts": o[1], "list_uploads": o[2], "blocks": o[3],
                "graphs_captured": o[4]}

    def stats(self):
        o = (C.c_int64 * 6)()
        _check(lib().w1_serve_stats(self.h, o), "w1_serve_stats")
        return {"admitted": o[0], "finished": o[1], "queued": o[2], "running": o[3], "bytes": o[4],
                "peak_bytes": o[5]}


# ---------------------------------------------------------------------------
# single-step entry points (device tensors; element type from precision)
# ---------------------------------------------------------------------------
def _dt(precision):
    return "float32" if precision == FP32 else "float64"


def op_prepare(n, levels, precision, p0, p1, rho_out, stream=None):
    ptrs = (C.c_void_p * levels)(*[_ptr(r, _dt(precision))[0] for r in rho_out])
    _check(lib().w1_op_prepare(n, levels, precision, _ptr(p0, "float64")[0], _ptr(p1, "float64")[0], ptrs,
                               _stream(stream)), "w1_op_prepare")


def op_prolong(nc, precision, c_m1, c_m2, c_phi, f_m1, f_m2, f_phi, stream=None):
    d = _dt(precision)
    _check(lib().w1_op_prolong(nc, precision, *[_ptr(x, d)[0] for x in (c_m1, c_m2, c_phi, f_m1, f_m2, f_phi)],
                               _stream(stream)), "w1_op_prolong")


def op_plain_steps(n, metric, precision, steps, m1, m2, phi, rho, step_scale=0.0, block_steps=0, fpr=False,
                   stream=None, waves=0, width=0, height=0):
    d = _dt(precision)
    out = C.c_double(np.nan)
    _check(lib().w1_op_plain_steps(n, metric, precision, step_scale, steps, block_steps, waves, width, height,
                                   *[_ptr(x, d)[0] for x in (m1, m2, phi, rho)],
                                   C.byref(out) if fpr else None, _stream(stream)), "w1_op_plain_steps")
    return out.value if fpr else None


def trim_cache() -> int:
    """Idle cached solve-state blocks back to the device; returns the bytes released."""
    out = C.c_size_t(0)
    _check(lib().w1_trim_cache(C.byref(out)), "w1_trim_cache")
    return int(out.value)


def tuner_table():
    """The launch-shape autotuner's measurements (list of dicts)."""
    import json
    n = lib().w1_tuner_table(None, 0)
    buf = C.create_string_buffer(n + 1)
    lib().w1_tuner_table(buf, n + 1)
    return json.loads(buf.value.decode())


def tuner_reset():
    _check(lib().w1_tuner_reset(), "w1_tuner_reset")


def op_prox_steps(n, metric, precision, steps, m1, m2, w1, w2, wb1, wb2, rho, step_scale=0.0, fpr=False,
                  stream=None, resident=False):
    d = _dt(precision)
    out = C.c_double(np.nan)
    _check(lib().w1_op_prox_steps(n, metric, precision, step_scale, steps, 1 if resident else 0,
                                  *[_ptr(x, d)[0] for x in (m1, m2, w1, w2, wb1, wb2, rho)],
                                  C.byref(out) if fpr else None, _stream(stream)), "w1_op_prox_steps")
    return out.value if fpr else None


def op_poisson(n, precision, r, u, stream=None):
    d = _dt(precision)
    _check(lib().w1_op_poisson(n, precision, _ptr(r, d)[0], _ptr(u, d)[0], _stream(stream)), "w1_op_poisson")


def op_poisson_noalloc(n, precision, r, u, stream=None):
    """w1_op_poisson without device allocation (static per-GPU working
    memory; asynchronous on `stream`)."""
    d = _dt(precision)
    _check(lib().w1_op_poisson_noalloc(n, precision, _ptr(r, d)[0], _ptr(u, d)[0], _stream(stream)),
           "w1_op_poisson_noalloc")


def noalloc_bytes():
    return int(lib().w1_noalloc_bytes())


def op_potential(n, precision, w1, w2, psi, stream=None):
    d = _dt(precision)
    _check(lib().w1_op_potential(n, precision, *[_ptr(x, d)[0] for x in (w1, w2, psi)], _stream(stream)),
           "w1_op_potential")


def op_evaluate(n, metric, precision, m1, m2, psi, rho, stream=None):
    d = _dt(precision)
    out = (C.c_double * 6)()
    _check(lib().w1_op_evaluate(n, metric, precision, *[_ptr(x, d)[0] for x in (m1, m2, psi, rho)], out,
                                _stream(stream)), "w1_op_evaluate")
    return {"P": out[0], "D": out[1], "lo": out[2], "hi": out[3], "kkt": out[4], "grad_max": out[5]}


def solve3d(p: Params, p0, p1, fields=False, stream=None):
    """Algorithm 3 or 4 (p.algo) in d = 3 on one pair of (n+1)^3 float64 masses (numpy or
    cuda tensors).  Returns the result dict, and with fields=True also
    (m, psi): m of shape (3, n+1, n+1, n+1) and psi (n+1, n+1, n+1), host."""
    pa, da = _ptr(p0, "float64")
    pb, db = _ptr(p1, "float64")
    if da != db:
        raise ValueError("both masses must be on the same side (host or device)")
    out = Result()
    n = p.n
    m = psi = None
    if fields:
        m = np.empty((3, n + 1, n + 1, n + 1))
        psi = np.empty((n + 1, n + 1, n + 1))
    _check(lib().w1_solve3d(C.byref(p), pa, pb, 1 if da else 0, C.byref(out),
                            m.ctypes.data if fields else None, psi.ctypes.data if fields else None,
                            _stream(stream)), "w1_solve3d")
    r = out.as_dict()
    return (r, m, psi) if fields else r


def op_plain_steps3d(n, metric, precision, steps, m1, m2, m3, phi, rho, step_scale=0.0, fpr=False, stream=None):
    d = _dt(precision)
    out = C.c_double(np.nan)
    _check(lib().w1_op_plain_steps3d(n, metric, precision, step_scale, steps,
                                     *[_ptr(x, d)[0] for x in (m1, m2, m3, phi, rho)],
                                     C.byref(out) if fpr else None, _stream(stream)), "w1_op_plain_steps3d")
    return out.value if fpr else None


def op_prox_steps3d(n, metric, precision, steps, m1, m2, m3, w1, w2, w3, wb1, wb2, wb3, rho, step_scale=0.0,
                    fpr=False, stream=None):
    d = _dt(precision)
    out = C.c_double(np.nan)
    _check(lib().w1_op_prox_steps3d(n, metric, precision, step_scale, steps,
                                    *[_ptr(x, d)[0] for x in (m1, m2, m3, w1, w2, w3, wb1, wb2, wb3, rho)],
                                    C.byref(out) if fpr else None, _stream(stream)), "w1_op_prox_steps3d")
    return out.value if fpr else None


def solve3d_batch(p: Params, pairs, workers=0):
    """w1_solve3d over a list of (p0, p1) pairs (all numpy or all cuda
    tensors) on `workers` concurrent streams; returns the result dicts."""
    k = len(pairs)
    A = (C.c_void_p * k)()
    B = (C.c_void_p * k)()
    dev = None
    for i, (a, b) in enumerate(pairs):
        pa, da = _ptr(a, "float64")
        pb, db = _ptr(b, "float64")
        if dev is None:
            dev = da
        if da != dev or db != dev:
            raise ValueError("all masses must be on the same side (host or device)")
        A[i], B[i] = pa, pb
    out = (Result * k)()
    _check(lib().w1_solve3d_batch(C.byref(p), k, A, B, 1 if dev else 0, out, workers), "w1_solve3d_batch")
    return [r.as_dict() for r in out]

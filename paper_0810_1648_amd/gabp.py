"""Python binding of the GaBP SVM C ABI (include/gabp_svm.h).

Argument marshalling only: every step of the solve runs in the HIP kernels
of libgabp_svm.so.  Inputs may be NumPy arrays (host memory) or torch CUDA
tensors (device memory, read on the current torch stream).  There is no
fallback: if the library is not built, or no gfx950 device is usable, the
calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgabp_svm.so")

# enums (mirrors of the header)
OK, E_INVALID, E_NOMEM, E_NOT_CONVERGED, E_DIVERGED, E_DEVICE, E_STATE, E_BUFSIZE = range(8)
KERNEL_RBF, KERNEL_PRECOMPUTED, KERNEL_RBF_SPARSE = 0, 2, 3
KERNEL = {"rbf": KERNEL_RBF, "precomputed": KERNEL_PRECOMPUTED, "rbf_sparse": KERNEL_RBF_SPARSE}
DIAG = {"none": 0, "softmargin": 1, "dominant_row": 2, "dominant_uniform": 3}
BOX = {"none": 0, "clip_output": 1, "project": 2}
PREC = {"fp64": 0, "fp32": 1, "mixed": 2}
KSTORE = {"auto": 0, "materialise": 1, "recompute": 2}
EDGE = {"auto": 0, "stored": 1, "stateless": 2}
GRAM = {"auto": 0, "bf16": 1, "bf16x3": 2, "bf16x6": 3}
SCHED = {"sync": 0, "grouped": 1}
MEM_HOST, MEM_DEVICE = 0, 1
REASON = {0: "none", 1: "converged", 2: "max_sweeps", 3: "diverged", 4: "stagnated"}
Q_N, Q_ALPHA, Q_PTILDE, Q_ADIAG, Q_BIAS, Q_SV_MASK, Q_SV_COUNT, Q_SWEEPS, Q_DELTA, Q_STATUS, \
    Q_TIMINGS, Q_TRACE, Q_PLAN, Q_REASON, Q_EDGES, Q_RESIDUAL_BOUND = range(16)


class Params(ct.Structure):
    _fields_ = [
        ("struct_size", ct.c_uint32), ("kernel", ct.c_int32), ("gamma", ct.c_double),
        ("C", ct.c_double), ("lambda_aug", ct.c_double), ("diag_mode", ct.c_int32),
        ("diag_delta", ct.c_double), ("box_mode", ct.c_int32), ("sv_tau", ct.c_double),
        ("tol_abs", ct.c_double), ("tol_rel", ct.c_double), ("max_sweeps", ct.c_int32),
        ("check_every", ct.c_int32), ("stagnation_window", ct.c_int32),
        ("stagnation_rel", ct.c_double), ("precision", ct.c_int32), ("kstore", ct.c_int32),
        ("edge_state", ct.c_int32), ("gram", ct.c_int32), ("stateless_depth", ct.c_int32),
        ("device", ct.c_int32), ("hbm_budget_bytes", ct.c_uint64), ("time_sweeps", ct.c_int32),
        ("schedule", ct.c_int32), ("sched_groups", ct.c_int32), ("sparse_edges_hint", ct.c_int32),
        ("sparse_tau", ct.c_double), ("tile_chunk", ct.c_int32),
    ]


class Timings(ct.Structure):
    _fields_ = [("stage_ms", ct.c_double), ("kbuild_ms", ct.c_double), ("diag_ms", ct.c_double),
                ("sweep_loop_ms", ct.c_double), ("sweep_kernel_ms", ct.c_double),
                ("sweep_launches", ct.c_int64), ("d2h_ms", ct.c_double), ("total_ms", ct.c_double),
                ("predict_kernel_ms", ct.c_double), ("predict_queries", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Plan(ct.Structure):
    _fields_ = [("precision", ct.c_int32), ("kstore", ct.c_int32), ("edge_state", ct.c_int32),
                ("gram", ct.c_int32), ("tile", ct.c_int32), ("stateless_depth", ct.c_int32),
                ("n_blocks", ct.c_int64), ("n_tiles", ct.c_int64), ("device_bytes", ct.c_uint64),
                ("alg_bytes_per_sweep", ct.c_uint64), ("alg_bytes_per_pair", ct.c_double),
                ("stateless_rho", ct.c_double), ("series_reciprocal", ct.c_int32), ("sched_groups", ct.c_int32),
                ("n_edges", ct.c_int64), ("stateless_bounded", ct.c_int32), ("tile_chunk", ct.c_int32),
                ("recompute_aug", ct.c_int32), ("reserved", ct.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GabpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None
ABI_VERSION = 9     # GABP_ABI_VERSION the structures above describe


def lib():
    """Loads libgabp_svm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
        L = ct.CDLL(LIB_PATH)
        vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
        L.gabp_svm_params_default.argtypes = [ct.POINTER(Params)]
        L.gabp_svm_params_default.restype = None
        L.gabp_svm_create.argtypes = [ct.POINTER(Params), ct.POINTER(vp)]
        L.gabp_svm_create.restype = i32
        L.gabp_svm_solve.argtypes = [vp, vp, vp, i64, i64, i32, vp]
        L.gabp_svm_solve.restype = i32
        L.gabp_svm_solve_kernel.argtypes = [vp, vp, vp, i64, i32, vp]
        L.gabp_svm_solve_kernel.restype = i32
        L.gabp_svm_query.argtypes = [vp, i32, vp, sz]
        L.gabp_svm_query.restype = i32
        L.gabp_svm_kernel_entries.argtypes = [vp, vp, vp, i64, vp]
        L.gabp_svm_kernel_entries.restype = i32
        L.gabp_svm_predict.argtypes = [vp, vp, i64, vp, i32, vp]
        L.gabp_svm_predict.restype = i32
        L.gabp_svm_predict_noalloc.argtypes = [vp, vp, i64, vp, vp]
        L.gabp_svm_predict_noalloc.restype = i32
        L.gabp_svm_destroy.argtypes = [vp]
        L.gabp_svm_destroy.restype = None
        L.gabp_status_string.argtypes = [i32]
        L.gabp_status_string.restype = ct.c_char_p
        L.gabp_svm_last_error.argtypes = [vp]
        L.gabp_svm_last_error.restype = ct.c_char_p
        L.gabp_abi_version.argtypes = []
        L.gabp_abi_version.restype = i32
        if L.gabp_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.gabp_abi_version()}, the binding expects "
                               f"{ABI_VERSION}: rebuild with __graft_entry__.build()")
        _lib = L
    return _lib


def default_params() -> Params:
    p = Params()
    lib().gabp_svm_params_default(ct.byref(p))
    return p


def make_params(**kw) -> Params:
    """Defaults of the library, overridden by keyword arguments; enum fields
    accept the lower-case names of the header (e.g. precision="fp32")."""
    p = default_params()
    maps = {"diag_mode": DIAG, "box_mode": BOX, "precision": PREC, "kstore": KSTORE,
            "edge_state": EDGE, "gram": GRAM, "schedule": SCHED}
    for k, v in kw.items():
        if k in maps and isinstance(v, str):
            v = maps[k][v]
        if k == "kernel" and isinstance(v, str):
            v = KERNEL[v]
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype):
    """(pointer, mem kind, keep-alive) for a NumPy array or torch tensor."""
    if _is_torch(x):
        import torch
        want = {np.float32: torch.float32, np.float64: torch.float64}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        return ct.c_void_p(x.data_ptr()), (MEM_DEVICE if x.is_cuda else MEM_HOST), x
    a = np.ascontiguousarray(x, dtype=dtype)
    return a.ctypes.data_as(ct.c_void_p), MEM_HOST, a


def _stream_of(x, stream):
    if stream is not None:
        return ct.c_void_p(int(stream))
    if _is_torch(x) and x.is_cuda:
        import torch
        return ct.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
    return ct.c_void_p(0)


class GabpSVM:
    """One solver handle (gabp_svm_create / solve / query / predict / destroy)."""

    def __init__(self, params: Params | None = None, **kw):
        self.params = params if params is not None else make_params(**kw)
        h = ct.c_void_p()
        st = lib().gabp_svm_create(ct.byref(self.params), ct.byref(h))
        if st != OK:
            raise GabpError(st, "gabp_svm_create failed: " + lib().gabp_status_string(st).decode())
        self._h = h
        self.last_status = None

    # -- lifecycle
    def close(self):
        if getattr(self, "_h", None):
            lib().gabp_svm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _err(self, st, what):
        msg = lib().gabp_svm_last_error(self._h).decode()
        return GabpError(st, f"{what}: {lib().gabp_status_string(st).decode()}: {msg}")

    # -- solves
    def solve(self, X, y, stream=None, raise_on=(E_INVALID, E_NOMEM, E_DEVICE, E_STATE)):
        """Runs gabp_svm_solve; returns the status code (OK, NOT_CONVERGED,
        DIVERGED) and raises on argument/device errors."""
        n, m = int(X.shape[0]), int(X.shape[1])
        px, mx, kx = _ptr(X, np.float32)
        py, my, ky = _ptr(y, np.float32)
        if mx != my:
            raise TypeError("X and y must live in the same memory")
        st = lib().gabp_svm_solve(self._h, px, py, n, m, mx, _stream_of(X, stream))
        del kx, ky
        self.last_status = st
        if st in raise_on:
            raise self._err(st, "gabp_svm_solve")
        return st

    def solve_kernel(self, K, y, stream=None, raise_on=(E_INVALID, E_NOMEM, E_DEVICE, E_STATE)):
        n = int(K.shape[0])
        pk, mk, kk = _ptr(K, np.float64)
        py, my, ky = _ptr(y, np.float32)
        if mk != my:
            raise TypeError("K and y must live in the same memory")
        st = lib().gabp_svm_solve_kernel(self._h, pk, py, n, mk, _stream_of(K, stream))
        del kk, ky
        self.last_status = st
        if st in raise_on:
            raise self._err(st, "gabp_svm_solve_kernel")
        return st

    # -- queries
    def _q(self, what, arr):
        st = lib().gabp_svm_query(self._h, what, arr.ctypes.data_as(ct.c_void_p), arr.nbytes)
        if st != OK:
            raise self._err(st, "gabp_svm_query")
        return arr

    def _qs(self, what, obj):
        st = lib().gabp_svm_query(self._h, what, ct.byref(obj), ct.sizeof(obj))
        if st != OK:
            raise self._err(st, "gabp_svm_query")
        return obj

    @property
    def n(self):
        return int(self._q(Q_N, np.zeros(1, np.int64))[0])

    def alpha(self):
        return self._q(Q_ALPHA, np.zeros(self.n))

    def ptilde(self):
        return self._q(Q_PTILDE, np.zeros(self.n))

    def adiag(self):
        return self._q(Q_ADIAG, np.zeros(self.n))

    def bias(self):
        return float(self._q(Q_BIAS, np.zeros(1))[0])

    def sv_mask(self):
        return self._q(Q_SV_MASK, np.zeros(self.n, np.uint8)).astype(bool)

    def sv_count(self):
        return int(self._q(Q_SV_COUNT, np.zeros(1, np.int64))[0])

    def sweeps(self):
        return int(self._q(Q_SWEEPS, np.zeros(1, np.int32))[0])

    def delta(self):
        return float(self._q(Q_DELTA, np.zeros(1))[0])

    def status(self):
        return int(self._q(Q_STATUS, np.zeros(1, np.int32))[0])

    def reason(self):
        return REASON[int(self._q(Q_REASON, np.zeros(1, np.int32))[0])]

    def trace(self):
        return self._q(Q_TRACE, np.zeros(self.sweeps()))

    def timings(self):
        return self._qs(Q_TIMINGS, Timings()).as_dict()

    def plan(self):
        return self._qs(Q_PLAN, Plan()).as_dict()

    def edges(self):
        """Kept pairs (i, j), i < j, of a sparsified solve (int64, E x 2)."""
        E = int(self.plan()["n_edges"])
        return self._q(Q_EDGES, np.zeros((E, 2), np.int64))

    def residual_bound(self):
        """GABP_Q_RESIDUAL_BOUND: ||1 - A alpha||_inf over all rows, the
        dominance gap min_i (A_ii - r_i) and Varah's bound on
        ||alpha - A^-1 1||_inf (one device pass over K')."""
        v = self._q(Q_RESIDUAL_BOUND, np.zeros(3))
        return {"residual_inf": float(v[0]), "gap": float(v[1]), "bound": float(v[2])}

    def kernel_entries(self, rows, cols):
        r = np.ascontiguousarray(rows, dtype=np.int64)
        c = np.ascontiguousarray(cols, dtype=np.int64)
        out = np.zeros(len(r))
        st = lib().gabp_svm_kernel_entries(self._h, r.ctypes.data_as(ct.c_void_p),
                                           c.ctypes.data_as(ct.c_void_p), len(r),
                                           out.ctypes.data_as(ct.c_void_p))
        if st != OK:
            raise self._err(st, "gabp_svm_kernel_entries")
        return out

    def predict(self, Xq, stream=None):
        nq = int(Xq.shape[0])
        px, mx, kx = _ptr(Xq, np.float32)
        if mx == MEM_DEVICE:
            import torch
            f = torch.empty(nq, dtype=torch.float64, device=Xq.device)
            pf = ct.c_void_p(f.data_ptr())
        else:
            f = np.zeros(nq)
            pf = f.ctypes.data_as(ct.c_void_p)
        st = lib().gabp_svm_predict(self._h, px, nq, pf, mx, _stream_of(Xq, stream))
        del kx
        if st != OK:
            raise self._err(st, "gabp_svm_predict")
        return f

    def predict_noalloc(self, Xq, f_out, stream=None):
        """gabp_svm_predict_noalloc: Xq (nq x m float32) and f_out (nq
        float64) are device tensors; the call only enqueues work on the
        stream (the tensors' current stream by default)."""
        nq = int(Xq.shape[0])
        px, mx, kx = _ptr(Xq, np.float32)
        pf, mf, kf = _ptr(f_out, np.float64)
        if mx != MEM_DEVICE or mf != MEM_DEVICE or int(f_out.shape[0]) != nq:
            raise TypeError("predict_noalloc takes device tensors Xq (nq x m) and f_out (nq)")
        st = lib().gabp_svm_predict_noalloc(self._h, px, nq, pf, _stream_of(Xq, stream))
        del kx, kf
        if st != OK:
            raise self._err(st, "gabp_svm_predict_noalloc")
        return f_out

# ------------------------------------------------------------------ serving --

class ServerParams(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("device", ct.c_int32), ("arena_bytes", ct.c_uint64),
                ("max_active", ct.c_int32), ("steps_per_poll", ct.c_int32), ("max_bypass", ct.c_int32),
                ("reserved", ct.c_int32)]


class RequestInfo(ct.Structure):
    _fields_ = [("status", ct.c_int32), ("reason", ct.c_int32), ("sweeps", ct.c_int32),
                ("stateless_levels", ct.c_int32), ("N", ct.c_int64), ("latency_ms", ct.c_double),
                ("queue_ms", ct.c_double), ("device_bytes", ct.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["reason"] = REASON.get(d["reason"], d["reason"])
        return d


class ServerStats(ct.Structure):
    _fields_ = [("submitted", ct.c_int64), ("completed", ct.c_int64), ("failed", ct.c_int64),
                ("p50_ms", ct.c_double), ("p99_ms", ct.c_double), ("mean_ms", ct.c_double),
                ("max_ms", ct.c_double), ("mean_queue_ms", ct.c_double), ("throughput_per_s", ct.c_double),
                ("mean_active", ct.c_double), ("max_active_seen", ct.c_int64), ("steps", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _server_lib():
    L = lib()
    if not getattr(L, "_server_ready", False):
        vp, i32, i64, u64p = ct.c_void_p, ct.c_int32, ct.c_int64, ct.POINTER(ct.c_uint64)
        L.gabp_server_params_default.argtypes = [ct.POINTER(ServerParams)]
        L.gabp_server_params_default.restype = None
        L.gabp_server_create.argtypes = [ct.POINTER(ServerParams), ct.POINTER(vp)]
        L.gabp_server_create.restype = i32
        L.gabp_server_submit.argtypes = [vp, vp, vp, i64, i64, ct.POINTER(Params), u64p]
        L.gabp_server_submit.restype = i32
        L.gabp_server_poll.argtypes = [vp, ct.c_uint64, ct.POINTER(i32)]
        L.gabp_server_poll.restype = i32
        L.gabp_server_wait.argtypes = [vp, ct.c_uint64, ct.c_double]
        L.gabp_server_wait.restype = i32
        L.gabp_server_result.argtypes = [vp, ct.c_uint64, vp, ct.c_size_t, ct.POINTER(RequestInfo)]
        L.gabp_server_result.restype = i32
        L.gabp_server_stats_get.argtypes = [vp, ct.POINTER(ServerStats)]
        L.gabp_server_stats_get.restype = i32
        L.gabp_server_destroy.argtypes = [vp]
        L.gabp_server_destroy.restype = None
        L._server_ready = True
    return L


class GabpServer:
    """Continuous-batching server (gabp_server_*): submit host arrays, poll,
    wait, fetch results and latency statistics."""

    def __init__(self, **kw):
        L = _server_lib()
        p = ServerParams()
        L.gabp_server_params_default(ct.byref(p))
        for k, v in kw.items():
            if not hasattr(p, k):
                raise TypeError(f"unknown server parameter {k!r}")
            setattr(p, k, v)
        h = ct.c_void_p()
        st = L.gabp_server_create(ct.byref(p), ct.byref(h))
        if st != OK:
            raise GabpError(st, "gabp_server_create failed: " + L.gabp_status_string(st).decode())
        self._h = h
        self._n = {}

    def close(self):
        if getattr(self, "_h", None):
            _server_lib().gabp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def submit(self, X, y, params: Params | None = None, **kw) -> int:
        p = params if params is not None else make_params(**kw)
        X = np.ascontiguousarray(X, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        t = ct.c_uint64()
        st = _server_lib().gabp_server_submit(self._h, X.ctypes.data_as(ct.c_void_p), y.ctypes.data_as(ct.c_void_p),
                                              X.shape[0], X.shape[1], ct.byref(p), ct.byref(t))
        if st != OK:
            raise GabpError(st, "gabp_server_submit: " + lib().gabp_status_string(st).decode())
        self._n[t.value] = X.shape[0]
        return t.value

    def poll(self, ticket) -> bool:
        d = ct.c_int32()
        st = _server_lib().gabp_server_poll(self._h, ticket, ct.byref(d))
        if st != OK:
            raise GabpError(st, "gabp_server_poll")
        return bool(d.value)

    def wait(self, ticket, timeout_s=-1.0) -> bool:
        return _server_lib().gabp_server_wait(self._h, ticket, timeout_s) == OK

    def result(self, ticket):
        a = np.zeros(self._n[ticket])
        info = RequestInfo()
        st = _server_lib().gabp_server_result(self._h, ticket, a.ctypes.data_as(ct.c_void_p), a.nbytes,
                                              ct.byref(info))
        if st != OK:
            raise GabpError(st, "gabp_server_result")
        return a, info.as_dict()

    def stats(self):
        s = ServerStats()
        st = _server_lib().gabp_server_stats_get(self._h, ct.byref(s))
        if st != OK:
            raise GabpError(st, "gabp_server_stats_get")
        return s.as_dict()

"""ctypes access to the compiled FP64 C oracle (test infrastructure only).

The shared object is built from gabp_oracle.c with gcc -O3 -mavx2 -fopenmp
and no fast-math or contraction (-ffp-contract=off keeps every product and
sum a separately rounded IEEE operation), by the repository's build step.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgabp_oracle.so")
SRC_PATH = os.path.join(_HERE, "gabp_oracle.c")

DIAG = {"none": 0, "softmargin": 1, "dominant_row": 2, "dominant_uniform": 3}
STATUS = {0: "converged", 3: "not_converged", 4: "diverged", 2: "nomem", 1: "invalid"}
CFLAGS = ["-O3", "-mavx2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU code involved)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        subprocess.check_call(["gcc", *CFLAGS, "-o", LIB_PATH, SRC_PATH, "-lm"])
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ct.CDLL(LIB_PATH)
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        L.oracle_svm_solve.argtypes = [f32p, f32p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                       ct.c_double, ct.c_int, ct.c_double, ct.c_int, ct.c_double,
                                       ct.c_double, f64p, f64p, f64p, f64p,
                                       ct.POINTER(ct.c_int), f64p]
        L.oracle_matrix_solve.argtypes = [f64p, f64p, ct.c_int64, ct.c_int, ct.c_double, ct.c_double,
                                          f64p, f64p, f64p, ct.POINTER(ct.c_int)]
        L.oracle_svm_residual_rows.argtypes = [f32p, f32p, ct.c_int64, ct.c_int64, ct.c_double,
                                               ct.c_double, ct.c_double, ct.c_int, ct.c_double, f64p,
                                               i64p, ct.c_int64, f64p, f64p]
        L.oracle_time_sweeps.argtypes = [f32p, f32p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                         ct.c_double, ct.c_int, ct.c_double, ct.c_int,
                                         ct.POINTER(ct.c_double), ct.POINTER(ct.c_int)]
        L.oracle_kernel_row.argtypes = [f32p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                        ct.c_int64, f64p]
        L.oracle_max_threads.restype = ct.c_int
        L.oracle_svm_matvec.argtypes = [f32p, f32p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                        ct.c_double, ct.c_int, ct.c_double, f64p, f64p, ct.c_void_p]
        L.oracle_stateless_matrix.argtypes = [f64p, f64p, ct.c_int64, ct.c_int, ct.c_int, f64p, f64p]
        L.oracle_stateless_rows.argtypes = [f32p, f32p, ct.c_int64, ct.c_int64, ct.c_double, ct.c_double,
                                            f64p, f64p, f64p, ct.c_int, ct.c_int, i64p, ct.c_int64,
                                            f64p, f64p, ct.POINTER(ct.c_double)]
        L.oracle_set_threads.argtypes = [ct.c_int]
        _lib = L
    return _lib


def svm_solve(X, y, gamma, C, lam, diag="dominant_row", delta=0.1, max_sweeps=1000,
              tol_abs=0.0, tol_rel=1e-12):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n, m = X.shape
    alpha = np.zeros(n)
    pt = np.zeros(n)
    adiag = np.zeros(n)
    deltas = np.zeros(max(max_sweeps, 1))
    timing = np.zeros(2)
    sw = ct.c_int(0)
    st = lib().oracle_svm_solve(X, y, n, m, gamma, C, lam, DIAG[diag], delta, max_sweeps, tol_abs,
                                tol_rel, alpha, pt, adiag, deltas, ct.byref(sw), timing)
    return dict(alpha=alpha, ptilde=pt, adiag=adiag, deltas=deltas[:sw.value], sweeps=sw.value,
                status=STATUS[st], build_s=timing[0], sweep_s=timing[1])


def matrix_solve(A, b, max_sweeps=1000, tol_abs=0.0, tol_rel=1e-12):
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(b)
    alpha = np.zeros(n)
    pt = np.zeros(n)
    deltas = np.zeros(max(max_sweeps, 1))
    sw = ct.c_int(0)
    st = lib().oracle_matrix_solve(A, b, n, max_sweeps, tol_abs, tol_rel, alpha, pt, deltas, ct.byref(sw))
    return dict(alpha=alpha, ptilde=pt, deltas=deltas[:sw.value], sweeps=sw.value, status=STATUS[st])


def residual_rows(X, y, gamma, C, lam, alpha, rows, diag="dominant_row", delta=0.1):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    alpha = np.ascontiguousarray(alpha, dtype=np.float64)
    n, m = X.shape
    res = np.zeros(len(rows))
    ad = np.zeros(len(rows))
    st = lib().oracle_svm_residual_rows(X, y, n, m, gamma, C, lam, DIAG[diag], delta, alpha, rows,
                                        len(rows), res, ad)
    if st != 0:
        raise RuntimeError(f"oracle_svm_residual_rows failed: {STATUS.get(st, st)}")
    return res, ad


def kernel_row(X, gamma, lam, i):
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, m = X.shape
    out = np.zeros(n)
    lib().oracle_kernel_row(X, n, m, gamma, lam, i, out)
    return out


def time_sweeps(X, y, gamma, C, lam, nsweeps, diag="dominant_row", delta=0.1):
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n, m = X.shape
    secs = ct.c_double(0.0)
    thr = ct.c_int(0)
    st = lib().oracle_time_sweeps(X, y, n, m, gamma, C, lam, DIAG[diag], delta, nsweeps,
                                  ct.byref(secs), ct.byref(thr))
    return dict(seconds=secs.value, threads=thr.value, status=STATUS[st])


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def svm_matvec(X, y, gamma, C, lam, v, diag="dominant_row", delta=0.1, want_diag=False):
    """A v for the SVM system without forming A (rows rebuilt from the
    features); with want_diag, also the weighted diagonal A_ii."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    v = np.ascontiguousarray(v, dtype=np.float64)
    n, m = X.shape
    out = np.zeros(n)
    ad = np.zeros(n) if want_diag else None
    st = lib().oracle_svm_matvec(X, y, n, m, gamma, C, lam, DIAG[diag], delta, v, out,
                                 ad.ctypes.data if want_diag else None)
    if st != 0:
        raise RuntimeError(f"oracle_svm_matvec failed: {STATUS.get(st, st)}")
    return (out, ad) if want_diag else out


def stateless_matrix(A, b, depth, sweeps):
    """Stateless-form trajectory alpha^1 .. alpha^sweeps on an explicit A."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(b)
    traj = np.zeros((sweeps, n))
    pt = np.zeros(n)
    st = lib().oracle_stateless_matrix(A, b, n, depth, sweeps, traj, pt)
    return dict(trajectory=traj, ptilde=pt, status=STATUS[st])


def stateless_rows(X, y, gamma, lam, adiag, hist_P, hist_S, t, depth, rows):
    """Aggregates (P~^t, S^t) of the listed rows after stateless sweep t of
    the SVM system; hist_P / hist_S are (t, N) aggregate histories."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    n, m = X.shape
    hist_P = np.ascontiguousarray(hist_P, dtype=np.float64)
    hist_S = np.ascontiguousarray(hist_S, dtype=np.float64)
    assert hist_P.shape == (t, n) and hist_S.shape == (t, n)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    outP = np.zeros(len(rows))
    outS = np.zeros(len(rows))
    secs = ct.c_double(0.0)
    st = lib().oracle_stateless_rows(X, y, n, m, gamma, lam, np.ascontiguousarray(adiag, dtype=np.float64),
                                     hist_P, hist_S, t, depth, rows, len(rows), outP, outS, ct.byref(secs))
    return dict(P=outP, S=outS, seconds=secs.value, status=STATUS[st])


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))

#!/usr/bin/env python3
"""Writes the FP64 reference solutions alpha* = A^-1 1 of the benchmark
workloads into tests/golden/alpha_ref/ (test infrastructure).

Only the seeded input generators (paper_0810_1648_amd/inputs.py, which hold
none of the solver's arithmetic) and the oracle (oracle/) are called.  For
every workload:

* A = weighted(Y K' Y) with the dominant-row diagonal (the system of section
  "Proposed Solution of SVM Solver Based on GaBP" with the weighting of
  subsection "GaBP Algorithm Convergence"), never formed: the oracle's
  matrix-free product rebuilds each row from the features in FP64;
* alpha* by Jacobi-preconditioned conjugate gradients to a relative residual
  of 1e-13;
* the certificate: the true residual r = 1 - A alpha* (one more product, with
  compensated sums) and Varah's bound ||alpha* - A^-1 1||_inf <=
  ||r||_inf / min_i (A_ii - sum_{j != i} |A_ij|), the row sums taken from
  A y (|A_ij| = y_i y_j A_ij);
* for the 20,000-point workload, also the oracle's own FP64 GaBP solve
  (Algorithm 2, stored messages, to 1e-13) and LAPACK Cholesky, both
  compared with alpha*.

Each file stores alpha (and, for the 100k workload, the weighted diagonal)
with the SHA-256 of the generated X and y, so a test can tell that it holds
the solution of the very arrays it generated.

    python tests/golden/make_alpha_ref.py tiny letter covertype serve large
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import gabp_ref as R  # noqa: E402
from oracle import oracle_c as oc  # noqa: E402
from paper_0810_1648_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "alpha_ref")
SERVE_IDS = list(range(8))      # the first requests of the serving stream (seed 3)


def data_sha256(X, y) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(X, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(y, dtype=np.float32).tobytes())
    return h.hexdigest()


def reference(wl, log_name, extra=None, keep_adiag=False, cross_check=False):
    t0 = time.time()
    mv = lambda v: oc.svm_matvec(wl.X, wl.y, wl.gamma, wl.C, wl.lam, v, delta=wl.delta)  # noqa: E731
    ones = np.ones(wl.N)
    _, adiag = oc.svm_matvec(wl.X, wl.y, wl.gamma, wl.C, wl.lam, ones, delta=wl.delta, want_diag=True)

    def log(it, rel):
        print(f"  [{log_name}] PCG iteration {it}: ||r|| / ||b|| = {rel:.3e} ({time.time() - t0:.0f} s)",
              flush=True)

    alpha, iters = R.pcg_solve(mv, ones, adiag, tol=1e-13, log=log)
    resid = ones - mv(alpha)
    yv = wl.y.astype(np.float64)
    rows = yv * mv(yv) - adiag                      # sum_{j != i} |A_ij|
    gap = float(np.min(adiag - rows))
    bound = float(np.max(np.abs(resid))) / gap if gap > 0 else float("inf")
    meta = {"workload": wl.name, "N": wl.N, "m": wl.m, "gamma": wl.gamma, "C": wl.C, "lam": wl.lam,
            "delta": wl.delta, "diag": "dominant_row", "data_sha256": data_sha256(wl.X, wl.y),
            "method": "Jacobi-preconditioned CG on the matrix-free FP64 oracle product, rel. residual 1e-13",
            "pcg_iterations": int(iters), "residual_inf": float(np.max(np.abs(resid))),
            "diag_gap_min": gap, "varah_bound_abs": bound,
            "varah_bound_rel": bound / float(np.max(np.abs(alpha))),
            "alpha_inf": float(np.max(np.abs(alpha))), "seconds": time.time() - t0}
    if cross_check:
        g = oc.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta, tol_rel=1e-13, max_sweeps=2000)
        meta["oracle_gabp"] = {"status": g["status"], "sweeps": g["sweeps"],
                               "rel_diff_vs_cg": float(np.max(np.abs(g["alpha"] - alpha)) / meta["alpha_inf"])}
        A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta)
        ch = R.cholesky_solve(A, b)
        del A
        meta["cholesky_rel_diff_vs_cg"] = float(np.max(np.abs(ch - alpha)) / meta["alpha_inf"])
        assert g["status"] == "converged" and meta["oracle_gabp"]["rel_diff_vs_cg"] < 1e-10
        assert meta["cholesky_rel_diff_vs_cg"] < 1e-11
    if extra:
        meta.update(extra)
    assert meta["varah_bound_rel"] < 1e-10, meta
    arrays = {"alpha": alpha}
    if keep_adiag:
        arrays["adiag"] = adiag
    return arrays, meta


def save(name, arrays, meta):
    os.makedirs(OUT, exist_ok=True)
    np.savez(os.path.join(OUT, f"{name}.npz"), **arrays)
    with open(os.path.join(OUT, f"{name}.json"), "w") as fh:
        json.dump(meta, fh, indent=1, sort_keys=True)
        fh.write("\n")
    print(f"wrote {name}: {json.dumps(meta)}", flush=True)


def main(names):
    for name in names:
        if name == "serve":
            stream = inputs.serving_stream(512, rate_per_s=1.0, seed=3)
            for rid in SERVE_IDS:
                wl = stream[rid].workload
                arrays, meta = reference(wl, f"serve req {rid}", extra={"request": rid, "stream_seed": 3})
                save(f"serve_req{rid}", arrays, meta)
        else:
            wl = inputs.make_workload(name)
            arrays, meta = reference(wl, name, keep_adiag=(name == "covertype"),
                                     cross_check=(name in ("tiny", "letter")))
            save(name, arrays, meta)


if __name__ == "__main__":
    main(sys.argv[1:] or ["tiny", "letter", "covertype", "serve", "large"])

"""The stored FP64 reference solutions alpha* (tests/golden/alpha_ref/,
written by tests/golden/make_alpha_ref.py from the oracle alone) are what the
oracle says they are, for the very arrays the generators produce now.

For every stored workload: the SHA-256 of the regenerated X and y matches the
one recorded with alpha*; the certificate recorded by the generating run
(Varah's bound from the true residual) is below 1e-10 relative; and residual
rows recomputed here by a different route (the oracle's row-at-a-time
kernel, direct FP64 differences) are at the level that certificate implies.
The tiny workload is checked against LAPACK Cholesky in full.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from oracle import gabp_ref as R
from paper_0810_1648_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alpha_ref")
KEYS = sorted(f[:-5] for f in os.listdir(GOLDEN) if f.endswith(".json")) if os.path.isdir(GOLDEN) else []


def _workload(key):
    if key.startswith("serve_req"):
        rid = int(key[len("serve_req"):])
        return inputs.serving_stream(rid + 1, rate_per_s=1.0, seed=3)[rid].workload
    return inputs.make_workload(key)


def test_references_exist():
    for key in ("tiny", "letter", "covertype", "large", "serve_req0"):
        assert key in KEYS, key


@pytest.mark.parametrize("key", KEYS)
def test_reference_is_the_oracle_solution(oracle_c, key):
    meta = json.load(open(os.path.join(GOLDEN, f"{key}.json")))
    alpha = np.load(os.path.join(GOLDEN, f"{key}.npz"))["alpha"]
    wl = _workload(key)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(wl.X, dtype=np.float32).tobytes())
    h.update(np.ascontiguousarray(wl.y, dtype=np.float32).tobytes())
    assert h.hexdigest() == meta["data_sha256"]
    assert meta["N"] == wl.N == len(alpha) and meta["m"] == wl.m
    assert (meta["gamma"], meta["C"], meta["lam"], meta["delta"]) == (wl.gamma, wl.C, wl.lam, wl.delta)
    assert meta["varah_bound_rel"] < 1e-10 and meta["diag_gap_min"] > 0
    rows = np.unique(np.concatenate([[0, wl.N - 1], np.random.default_rng(1).choice(wl.N, 10, replace=False)]))
    res, ad = oracle_c.residual_rows(wl.X, wl.y, wl.gamma, wl.C, wl.lam, alpha, rows, delta=wl.delta)
    # a residual of the certified size: |r_i| <= ||r||_inf recorded (to rounding)
    assert np.max(np.abs(res)) <= 2.0 * meta["residual_inf"] + 1e-14 * np.max(ad * np.abs(alpha[rows]))
    if key == "tiny":
        A, b = R.svm_system(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta)
        exact = R.cholesky_solve(A, b)
        assert np.max(np.abs(alpha - exact)) <= 1e-12 * np.max(np.abs(exact))
    if key in ("tiny", "letter"):
        assert meta["oracle_gabp"]["status"] == "converged"
        assert meta["oracle_gabp"]["rel_diff_vs_cg"] < 1e-10 and meta["cholesky_rel_diff_vs_cg"] < 1e-11

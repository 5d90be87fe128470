"""Served form: continuous batching of many solves.

Each request's alpha must equal the single-handle solve of the same problem
bitwise (same kernels, same per-request reduction order), whether the
request runs alone or in a mix of uneven sizes and precisions; the
tolerance stated for serving (1e-5 relative to the FP64 oracle) then
follows from the single-solve parity tests.
"""
import json
import os
import time

import numpy as np
import pytest

from oracle import gabp_ref as R
from paper_0810_1648_amd import gabp, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _mix(n_req, seed, n_min=200, n_max=2600):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(n_req):
        n = int(np.exp(rng.uniform(np.log(n_min), np.log(n_max))))
        m = int(rng.choice([8, 32, 128]))
        C = float(rng.choice([0.1, 1.0, 10.0]))
        prec = ["fp32", "mixed", "fp64"][r % 3]
        X, y = inputs.blobs(n, m, 5000 + r)
        out.append((X, y, dict(gamma=1.0 / m, C=C, precision=prec, tol_rel=1e-7, edge_state="stored",
                               kstore="materialise")))
    return out


def _single(X, y, kw):
    s = gabp.GabpSVM(**kw)
    st = s.solve(X, y)
    a = s.alpha()
    sw = s.sweeps()
    s.close()
    return st, a, sw


def test_served_equals_single_alone_and_in_mix(torch):
    reqs = _mix(12, seed=1)
    print(f"[case] serving mix of {len(reqs)} requests, N {[r[0].shape[0] for r in reqs]}", flush=True)
    single = [_single(X, y, kw) for X, y, kw in reqs]
    # alone: one request per fresh server
    with gabp.GabpServer(arena_bytes=int(2e9), max_active=8) as srv:
        t = srv.submit(reqs[4][0], reqs[4][1], **reqs[4][2])
        assert srv.wait(t, 120.0)
        alone, info = srv.result(t)
    assert np.array_equal(alone, single[4][1])
    # in a mix, all submitted at once (more requests than slots)
    with gabp.GabpServer(arena_bytes=int(2e9), max_active=5, steps_per_poll=3) as srv:
        tickets = [srv.submit(X, y, **kw) for X, y, kw in reqs]
        for t in tickets:
            assert srv.wait(t, 300.0)
        for k, t in enumerate(tickets):
            a, info = srv.result(t)
            st, ref, sw = single[k]
            assert info["status"] == st and info["sweeps"] == sw, (k, info, st, sw)
            assert np.array_equal(a, ref), k
        stats = srv.stats()
    print("serving stats", stats)
    assert stats["completed"] + stats["failed"] == len(reqs)
    assert 1 <= stats["max_active_seen"] <= 5
    assert stats["p50_ms"] <= stats["p99_ms"] <= stats["max_ms"]


def test_served_result_matches_oracle(torch):
    X, y = inputs.blobs(900, 16, 31)
    with gabp.GabpServer(arena_bytes=int(1e9)) as srv:
        t = srv.submit(X, y, gamma=1.0 / 16, C=1.0, precision="mixed", tol_rel=1e-9)
        assert srv.wait(t, 120.0)
        a, info = srv.result(t)
    A, b = R.svm_system(X, y, 1.0 / 16, 1.0, 1.0 / 900)
    exact = R.cholesky_solve(A, b)
    err = float(np.max(np.abs(a - exact)) / np.max(np.abs(exact)))
    print(f"served mixed N=900: sweeps {info['sweeps']} rel err {err:.2e}")
    assert info["status"] == gabp.OK and err <= 1e-5


def test_admission_by_footprint(torch):
    # arena sized for about two of these requests at a time
    reqs = _mix(6, seed=3, n_min=1500, n_max=1600)
    reqs = [(X, y, dict(kw, precision="fp32")) for X, y, kw in reqs]
    one = 5 * 21 * 65536 * 4   # five FP32 planes of a 6-block problem (21 tiles)
    with gabp.GabpServer(arena_bytes=int(2.6 * one), max_active=8) as srv:
        tickets = [srv.submit(X, y, **kw) for X, y, kw in reqs]
        for t in tickets:
            assert srv.wait(t, 300.0)
        stats = srv.stats()
        infos = [srv.result(t)[1] for t in tickets]
    print("admission stats", stats)
    assert stats["max_active_seen"] <= 2
    assert all(i["status"] == gabp.OK for i in infos)
    with gabp.GabpServer(arena_bytes=int(0.5 * one)) as srv:
        with pytest.raises(gabp.GabpError) as e:
            srv.submit(reqs[0][0], reqs[0][1], **reqs[0][2])
        assert e.value.status == gabp.E_NOMEM


def test_served_stateless_plans_equal_single(torch):
    # edge state chosen per request from the contraction bound (AUTO): the
    # stateless requests run in launches grouped by precision and level
    # count, next to stored ones, and still match the single solve bitwise
    reqs = []
    for r in range(9):
        n = [300, 700, 1300][r % 3]
        X, y = inputs.blobs(n, 16, 7100 + r)
        gamma = [2e-3, 1.0 / 16, 0.5][r % 3]        # from strongly to weakly contracting
        prec = ["fp32", "mixed", "fp64"][(r // 3) % 3]
        # every other request asks for 2 x 2 tile chunks (taken where its plan
        # allows them), next to requests on single tiles in the same launches
        reqs.append((X, y, dict(gamma=gamma, C=1.0, precision=prec, tol_rel=1e-7, kstore="materialise",
                                tile_chunk=2 * (r % 2))))
    # shallow explicit recursions whose plans allow chunks: one level (FP32),
    # two levels with series reciprocals (MIXED)
    for r, (prec, depth) in enumerate((("fp32", 1), ("mixed", 2))):
        X, y = inputs.blobs([700, 1300][r], 16, 7150 + r)
        reqs.append((X, y, dict(gamma=2e-3, C=1.0, precision=prec, tol_rel=1e-7, kstore="materialise",
                                edge_state="stateless", stateless_depth=depth, tile_chunk=2)))
    print(f"[case] stateless serving mix of {len(reqs)} requests", flush=True)
    single, chunks = [], []
    for X, y, kw in reqs:
        s = gabp.GabpSVM(**kw)
        st = s.solve(X, y)
        single.append((st, s.alpha(), s.sweeps(), s.plan()["stateless_depth"]))
        chunks.append(s.plan()["tile_chunk"])
        s.close()
    levels = [d for _, _, _, d in single]
    print("single-solve levels", levels, "tile chunks", chunks)
    assert 2 in chunks and 1 in chunks
    assert any(d > 0 for d in levels) and len(set(levels)) >= 2
    with gabp.GabpServer(arena_bytes=int(2e9), max_active=6, steps_per_poll=2) as srv:
        tickets = [srv.submit(X, y, **kw) for X, y, kw in reqs]
        for t in tickets:
            assert srv.wait(t, 300.0)
        for k, t in enumerate(tickets):
            a, info = srv.result(t)
            st, ref, sw, d = single[k]
            assert info["stateless_levels"] == d, (k, info, d)
            assert info["status"] == st and info["sweeps"] == sw, (k, info, st, sw)
            assert np.array_equal(a, ref), k


def test_served_grouped_schedule_equals_single(torch):
    # GROUPED requests advance one group visit per step and must match the
    # single grouped solve bitwise, with stateless plans and with stored pair
    # records, alone and next to synchronous requests
    reqs = []
    for r in range(8):
        n = [200, 900, 2100, 4700][r % 4]             # 1 to 19 blocks
        X, y = inputs.blobs(n, 16, 7300 + r)
        gamma = [2e-3, 1.0 / 16, 0.5][r % 3]          # 0.5: stored pair records
        prec = ["fp32", "mixed", "fp64"][(r // 3) % 3]
        kw = dict(gamma=gamma, C=1.0, precision=prec, tol_rel=1e-7, kstore="materialise",
                  schedule="grouped", sched_groups=[0, 3][r % 2])
        reqs.append((X, y, kw))
    reqs.append((reqs[1][0], reqs[1][1], dict(reqs[1][2], schedule="sync")))
    reqs.append((reqs[5][0], reqs[5][1], dict(reqs[5][2], schedule="sync")))
    print(f"[case] grouped serving mix of {len(reqs)} requests", flush=True)
    single = []
    for X, y, kw in reqs:
        s = gabp.GabpSVM(**kw)
        st = s.solve(X, y)
        d = s.plan()["stateless_depth"]
        single.append((st, s.alpha(), s.sweeps(), d))
        s.close()
    print("single-solve levels", [d for *_, d in single], "sweeps", [sw for _, _, sw, _ in single])
    grouped_levels = [d for (X, y, kw), (_, _, _, d) in zip(reqs, single) if kw["schedule"] == "grouped"]
    assert sum(d > 0 for d in grouped_levels) >= 3 and sum(d == 0 for d in grouped_levels) >= 1
    with gabp.GabpServer(arena_bytes=int(2e9), max_active=1) as srv:
        t = srv.submit(reqs[2][0], reqs[2][1], **reqs[2][2])
        assert srv.wait(t, 120.0)
        alone, info = srv.result(t)
    assert info["sweeps"] == single[2][2] and np.array_equal(alone, single[2][1])
    with gabp.GabpServer(arena_bytes=int(2e9), max_active=6, steps_per_poll=3) as srv:
        tickets = [srv.submit(X, y, **kw) for X, y, kw in reqs]
        for t in tickets:
            assert srv.wait(t, 300.0)
        for k, t in enumerate(tickets):
            a, info = srv.result(t)
            st, ref, sw, d = single[k]
            assert info["status"] == st and info["sweeps"] == sw, (k, info, st, sw)
            assert np.array_equal(a, ref), k


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alpha_ref")


@pytest.mark.parametrize("precision", ["fp32", "mixed"])
def test_served_stream_matches_alpha_ref(torch, precision):
    """The first requests of the benchmark's serving stream (seed 3), served
    together, against the oracle's alpha* of each (conjugate gradients on the
    FP64 matrix-free product; tests/golden/alpha_ref/serve_req*.npz), element
    by element: ||alpha - alpha*||_inf <= 1e-5 ||alpha*||_inf, in FP32 and in
    the mixed precision pattern."""
    import hashlib
    stream = inputs.serving_stream(512, rate_per_s=1.0, seed=3)
    reqs = []
    for rid in range(8):
        meta = json.load(open(os.path.join(GOLDEN, f"serve_req{rid}.json")))
        wl = stream[rid].workload
        h = hashlib.sha256()
        h.update(wl.X.tobytes())
        h.update(wl.y.tobytes())
        assert meta["request"] == rid and h.hexdigest() == meta["data_sha256"]
        reqs.append((wl, np.load(os.path.join(GOLDEN, f"serve_req{rid}.npz"))["alpha"]))
    print(f"[case] served stream requests 0-7 ({precision}), N {[w.N for w, _ in reqs]}", flush=True)
    with gabp.GabpServer(arena_bytes=int(40e9), max_active=8) as srv:
        tickets = [srv.submit(wl.X, wl.y, gamma=wl.gamma, C=wl.C, precision=precision, tol_rel=wl.tol_rel,
                              kstore="materialise", schedule="grouped", sched_groups=4) for wl, _ in reqs]
        for t in tickets:
            assert srv.wait(t, 300.0)
        errs = []
        for (wl, ref), t in zip(reqs, tickets):
            a, info = srv.result(t)
            assert info["status"] == gabp.OK
            errs.append(float(np.max(np.abs(a - ref)) / np.max(np.abs(ref))))
    print(f"served {precision}: rel err vs alpha* per request {['%.1e' % e for e in errs]}")
    assert max(errs) <= 1e-5


def _footprint(X, y, kw):
    with gabp.GabpServer(arena_bytes=int(20e9), max_active=1) as srv:
        t = srv.submit(X, y, **kw)
        assert srv.wait(t, 120.0)
        return srv.result(t)[1]["device_bytes"]


def test_admission_fifo_with_bounded_bypass(torch):
    """Admission is FIFO with a bounded bypass: while a large request at the
    head of the queue does not fit, smaller requests behind it that fit are
    admitted, but at most max_bypass of them; later ones wait until the head
    has been admitted, and requests of equal size keep their submission
    order."""
    kwb = dict(gamma=1.0 / 16, C=1.0, precision="fp64", tol_rel=1e-12, edge_state="stored", kstore="materialise")
    kws = dict(gamma=1.0 / 16, C=1.0, precision="fp32", tol_rel=1e-7, edge_state="stored", kstore="materialise")
    big = [inputs.blobs(12000, 16, 8100 + k) for k in range(2)]
    small = [inputs.blobs(700, 16, 8200 + k) for k in range(5)]
    fb, fs = _footprint(*big[0], kwb), _footprint(*small[0], kws)
    print(f"[case] bypass: big footprint {fb / 1e9:.3f} GB, small {fs / 1e6:.1f} MB", flush=True)
    arena = int(fb + 3.5 * fs)          # one big request and three small ones at a time
    with gabp.GabpServer(arena_bytes=arena, max_active=16, max_bypass=2, steps_per_poll=1) as srv:
        sub = {}
        tickets = []
        for name, (X, y), kw in [("B0", big[0], kwb), ("B1", big[1], kwb)] + \
                [(f"s{k}", small[k], kws) for k in range(5)]:
            sub[name] = time.monotonic()
            tickets.append((name, srv.submit(X, y, **kw)))
        for _, t in tickets:
            assert srv.wait(t, 300.0)
        admit = {}
        for name, t in tickets:
            _, info = srv.result(t)
            assert info["status"] == gabp.OK, (name, info)
            admit[name] = sub[name] + info["queue_ms"] / 1e3
    order = sorted(admit, key=admit.get)
    print("admission order", order, {k: round((v - admit['B0']) * 1e3, 2) for k, v in admit.items()})
    eps = 2e-3                            # host clock reads around the submit calls
    # the head B1 waits for B0; two small requests pass it, the third does not
    assert admit["s0"] < admit["B1"] and admit["s1"] < admit["B1"]
    for k in (2, 3, 4):
        assert admit[f"s{k}"] >= admit["B1"] - eps, k
    for k in range(4):
        assert admit[f"s{k}"] <= admit[f"s{k + 1}"] + eps, k

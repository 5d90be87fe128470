#!/usr/bin/env python3
"""Benchmark of the GaBP SVM hot path on one MI355X.

A step is one full solve (staging, K' build, diagonal weighting, sweeps to
the stop rule, alpha download) of the covertype-shaped workload: N = 100k
points, m = 54 features (43 uniform + 11 one-hot), RBF gamma = 0.5, C = 1,
labels from a random RBF teacher with 5% flips, inputs resident in device
memory before the timed region.  The headline `value` is GaBP sweeps per
second over the whole timed job (all sweeps of all steps / wall time); the
same line carries solves/s, the error of every form against the oracle's
FP64 alpha* (tests/golden/alpha_ref/), the device's residual certificate,
the plain-FP32, stored-record, grouped, 20k-point (plain FP32) and
300k-point (K' recomputed) forms, the served stream in FP32 and in the mixed
pattern, the roofline of the sweep kernel and the timed CPU oracle.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
    python bench.py --ingest-counters FETCH_DIR WRITE_DIR   (writes profiles/sweep_traffic.json)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# VALU issue slots: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (FP32 and FP64 FMA
# both issue at one lane-op per lane per clock on CDNA4; packed FP32 unused)
VALU_PEAK_GSLOT = 256 * 64 * 2.4
# dense MFMA peaks (MI355X, no sparsity)
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "f32": 157.3}
# K' of one pair recomputed inside the sweep, beyond the MFMA Gram: the
# distance (norm sum, -2 g, clamp: 3), the scale (1), exp2 (a transcendental:
# 4) and + lambda^2 (1); from augmented rows, whose Gram is the exponent, the
# clamp (1), exp2 (4) and + lambda^2 (1)
RECOMPUTE_SLOTS_PER_PAIR = 9
RECOMPUTE_AUG_SLOTS_PER_PAIR = 6


def recompute_slots(plan):
    """VALU slots per pair of K' recomputed in the sweep (the plan's form)."""
    return RECOMPUTE_AUG_SLOTS_PER_PAIR if plan.get("recompute_aug", 0) else RECOMPUTE_SLOTS_PER_PAIR
# decision function on augmented rows (the MFMA emits the scaled exponent),
# VALU slots per (query, training point) pair: exp2 with its clamp modifier
# (a transcendental: 4 slots) and the FP32 multiply-add of the weighted sum
PREDICT_SLOTS_PER_PAIR = 5


# The sources of the kernels whose counter traffic is stored (the dense
# sweeps, the grouped visit and the K' build, MIXED path).
TRAFFIC_SOURCES = ("gabp_device.h", "gabp_internal.h", "gabp_kernels.hip", "gabp_sweep_mixed.hip")


def device_source_hash():
    """SHA-256 over the sources of the kernels whose traffic is stored (in
    name order)."""
    import hashlib
    d = os.path.join(ROOT, "paper_0810_1648_amd", "csrc")
    h = hashlib.sha256()
    for fn in sorted(TRAFFIC_SOURCES):
        h.update(fn.encode())
        h.update(open(os.path.join(d, fn), "rb").read())
    return h.hexdigest()


def stateless_slots_per_pair(levels, series, precision="mixed"):
    """Algorithmic VALU issue slots per pair of one stateless sweep with
    `levels` unrolled levels (both directions of the pair), counting a
    multiply-add as one slot (contracted, as the compiler emits it) and a
    transcendental as four.
    Series reciprocals (`series`: 1 / 2 terms at the top level, 3 = one term
    at the top and none at the lower levels; MIXED computes these messages
    in FP32 from FP32 K', so no conversion): a^2 (1); the lower levels carry
    G = P / (-a^2) and F = E / a: the deepest level is G = 1/P~, F = -S/P~ of
    its source (free), each middle level forms, per direction, a^2 u^2 (1)
    and G = u - a^2 u^2 G_rev (1) (not with series 3, where G = u),
    a F_rev - S (1) and F (1): 8 (4); the top level forms, per direction,
    the reciprocal u - a^2 u^2 G_rev (2: a^2 u^2, then one multiply-add;
    two terms: e = -a^2 G_rev u (2) and the series (2)), the accumulation
    of P (1, fused), a G (1), a F_rev - S (1) and the accumulation of E (1,
    fused): 12 (16 with two terms).  With one level the top level runs from
    zero reverse messages: 7.
    Exact reciprocals: per direction and level the cavity precision (1), the
    reciprocal (FP32: 4; FP64: 4 + two Newton steps of 2 FMAs = 8) and the
    messages (4; 3 at the top, where the accumulations fuse); MIXED adds the
    conversion of K' to FP64 (1)."""
    series = int(series)
    if series:
        if levels <= 1:
            return 7
        middle = 4 if series == 3 else 8
        top = 16 if series == 2 else 12
        return 1 + middle * (levels - 2) + top
    cvt = 1 if precision == "mixed" else 0
    r_top = 4 if precision == "fp32" else 8
    r_low = 8 if precision == "fp64" else 4
    return cvt + 1 + 2 * (levels - 1) * (1 + r_low + 4) + 2 * (1 + r_top + 3)


GOLDEN = os.path.join(ROOT, "tests", "golden", "alpha_ref")


def alpha_ref(key, X, y):
    """The oracle's FP64 alpha* for a workload (written by
    tests/golden/make_alpha_ref.py), or None when absent or computed from
    other arrays."""
    import hashlib

    import numpy as np
    try:
        meta = json.load(open(os.path.join(GOLDEN, f"{key}.json")))
        h = hashlib.sha256()
        h.update(np.ascontiguousarray(X, dtype=np.float32).tobytes())
        h.update(np.ascontiguousarray(y, dtype=np.float32).tobytes())
        if h.hexdigest() != meta["data_sha256"]:
            return None
        return np.load(os.path.join(GOLDEN, f"{key}.npz"))
    except (OSError, KeyError, ValueError):
        return None


def rel_err(a, ref):
    import numpy as np
    if ref is None:
        return None
    return float(np.max(np.abs(np.asarray(a) - ref)) / np.max(np.abs(ref)))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="covertype", choices=["covertype", "letter", "tiny", "large"])
    ap.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--gram", default="auto", choices=["auto", "bf16", "bf16x3", "bf16x6"])
    ap.add_argument("--kstore", default="auto", choices=["materialise", "recompute", "auto"])
    ap.add_argument("--edge", default="auto", choices=["stored", "stateless", "auto"])
    ap.add_argument("--no-stored", action="store_true", help="skip the stored-state (HBM-bound) comparison")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=0, help="oracle sample size (0 = auto)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-predict", action="store_true", help="skip the held-out decision-function measurement")
    ap.add_argument("--no-grouped", action="store_true", help="skip the grouped-schedule solve")
    ap.add_argument("--no-sparse", action="store_true", help="skip the sparsified-kernel solve")
    ap.add_argument("--sparse-n", type=int, default=1000000)
    ap.add_argument("--sparse-tau", type=float, default=0.55)
    ap.add_argument("--predict-n", type=int, default=100000, help="held-out queries of the predict leg")
    ap.add_argument("--serve-only", action="store_true", help="run only the serving measurement")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-load", type=float, default=0.8, help="offered load / measured capacity")
    ap.add_argument("--serve-precision", default="fp32", choices=["fp32", "mixed", "fp64"])
    ap.add_argument("--serve-steps-per-poll", type=int, default=2, help="server steps between status reads")
    ap.add_argument("--serve-groups", type=int, default=4,
                    help="groups of a served grouped request (0 = 16); a step visits one group of every request")
    ap.add_argument("--serve-schedule", default="grouped", choices=["grouped", "sync"],
                    help="schedule of the served requests (the other one is measured beside it)")
    ap.add_argument("--calib-copy-gb", type=float, default=0.0,
                    help="also run a plain device copy of this many GB (counter calibration)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "sweep_traffic.json"))
    ap.add_argument("--side-steps", type=int, default=2,
                    help="timed solves of the comparison legs (stored records, 20k and 300k workloads)")
    ap.add_argument("--no-letter", action="store_true", help="skip the 20k-point plain FP32 leg")
    ap.add_argument("--no-large", action="store_true", help="skip the 300k-point recompute leg")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="target seconds of each CPU-oracle sample")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE) of this benchmark into the "
                         "traffic JSON and exit")
    return ap.parse_args()


def solve_steps(torch, gabp, wl, X, y, params, steps, warmup, certificate=False):
    s = gabp.GabpSVM(**params)
    for _ in range(warmup):
        s.solve(X, y)
    torch.cuda.synchronize()
    sweeps = 0
    ktime = 0.0
    klaunch = 0
    t0 = time.perf_counter()
    for _ in range(steps):
        st = s.solve(X, y)
        sweeps += s.sweeps()
        tm = s.timings()
        ktime += tm["sweep_kernel_ms"]
        klaunch += tm["sweep_launches"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    info = dict(status=int(st), reason=s.reason(), sweeps_per_solve=s.sweeps(), plan=s.plan(),
                timings=s.timings(), alpha=s.alpha())
    if certificate:
        # outside the timed region: one pass over K' for ||1 - A alpha||_inf
        c = s.residual_bound()
        c["bound_rel"] = c["bound"] / float(abs(info["alpha"]).max())
        info["certificate"] = c
    s.close()
    return wall, sweeps, ktime, klaunch, info


def serving_bench(gabp, inputs, n_req, load, precision, schedule="grouped", seq_sample=24, steps_per_poll=2,
                  groups=0):
    """Serving stream: N log-uniform in [1k, 16k], m in {8, 32, 128}, C in
    {0.1, 1, 10}, two-blob data with per-request seed, gamma = 1/m, every
    request with the given schedule (grouped: stateless plans visit one group
    per step, stored plans run synchronously).  First the closed-loop
    capacity (all requests queued at once), then an open loop with Poisson
    arrivals at `load` x capacity for the latency percentiles, then
    sequential single solves of a sample for comparison (seq_sample > 0)."""
    import numpy as np
    stream = inputs.serving_stream(n_req, rate_per_s=1.0, seed=3)
    kws = [dict(gamma=r.workload.gamma, C=r.workload.C, precision=precision, tol_rel=r.workload.tol_rel,
                kstore="materialise", edge_state="auto", schedule=schedule, sched_groups=groups) for r in stream]
    sp = dict(arena_bytes=int(120e9), max_active=64, steps_per_poll=steps_per_poll)
    # closed loop
    with gabp.GabpServer(**sp) as srv:
        t0 = time.perf_counter()
        tickets = [srv.submit(r.workload.X, r.workload.y, **kw) for r, kw in zip(stream, kws)]
        for t in tickets:
            srv.wait(t)
        cap_wall = time.perf_counter() - t0
        closed = srv.stats()
        results = [srv.result(t) for t in tickets]
        infos = [r[1] for r in results]
    # error against the oracle's alpha* for the requests that have one
    errs = {}
    for r, (a, _) in zip(stream, results):
        ref = alpha_ref(f"serve_req{r.rid}", r.workload.X, r.workload.y)
        if ref is not None:
            errs[r.rid] = rel_err(a, ref["alpha"])
        sweeps = [i["sweeps"] for i in infos]
        plan_mix = {}
        for i in infos:
            key = "stored" if i["stateless_levels"] == 0 else f"stateless_{i['stateless_levels']}"
            plan_mix[key] = plan_mix.get(key, 0) + 1
    capacity = n_req / cap_wall
    print(f"[bench] serving ({schedule}) closed loop: {n_req} solves in {cap_wall:.2f} s", file=sys.stderr, flush=True)
    # open loop, Poisson arrivals at load x capacity
    rate = load * capacity
    rng = np.random.default_rng(11)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=n_req))
    with gabp.GabpServer(**sp) as srv:
        t0 = time.perf_counter()
        tickets = []
        for r, kw, ta in zip(stream, kws, arrivals):
            dt = ta - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(dt)
            tickets.append(srv.submit(r.workload.X, r.workload.y, **kw))
        for t in tickets:
            srv.wait(t)
        open_wall = time.perf_counter() - t0
        opened = srv.stats()
    print(f"[bench] serving ({schedule}) open loop at {rate:.1f}/s: {open_wall:.2f} s", file=sys.stderr, flush=True)
    # sequential single solves (one handle, one request at a time) on a sample
    k = min(seq_sample, n_req)
    seq_rate = None
    if k > 0:
        t0 = time.perf_counter()
        for r, kw in zip(stream[:k], kws[:k]):
            h = gabp.GabpSVM(**kw)
            h.solve(r.workload.X, r.workload.y)
            h.close()
        seq_wall = time.perf_counter() - t0
        work_all = sum(r.workload.N ** 2 for r in stream)
        work_k = sum(r.workload.N ** 2 for r in stream[:k])
        seq_rate = k / seq_wall * (work_k / k) / (work_all / n_req)
    return {"requests": n_req, "precision": precision, "schedule": schedule, "sched_groups": groups,
            "N_range": [int(min(r.workload.N for r in stream)), int(max(r.workload.N for r in stream))],
            "capacity_solves_per_s": capacity, "offered_rate_per_s": rate, "load": load,
            "p50_ms": opened["p50_ms"], "p99_ms": opened["p99_ms"], "mean_ms": opened["mean_ms"],
            "max_ms": opened["max_ms"], "mean_queue_ms": opened["mean_queue_ms"],
            "throughput_solves_per_s": opened["throughput_per_s"],
            "mean_active": opened["mean_active"], "max_active_seen": opened["max_active_seen"],
            "closed_loop_p50_ms": closed["p50_ms"], "closed_loop_p99_ms": closed["p99_ms"],
            "mean_sweeps": float(np.mean(sweeps)), "plan_mix": plan_mix,
            "failed": opened["failed"] + closed["failed"],
            "err_vs_oracle": {"requests": sorted(errs), "max_rel": max(errs.values()) if errs else None,
                              "per_request": [errs[k] for k in sorted(errs)],
                              "note": "||alpha - alpha*||_inf / ||alpha*||_inf of the served results (closed "
                                      "loop) against the oracle's FP64 alpha* of the same requests"},
            "sequential_solves_per_s_est": seq_rate,
            "sequential_sample": (f"first {k} requests solved one at a time on one handle, rate scaled by "
                                  f"the stream's mean N^2 over the sample's") if k > 0 else None,
            "batching_speedup": capacity / seq_rate if seq_rate else None}


def predict_bench(torch, gabp, inputs, wl, X, y, params, n_test, reps=5):
    """Decision function of the trained machine on n_test held-out points of
    the same generator and teacher (device-resident queries): predictions/s
    over the whole call, the decision kernel's own time, held-out accuracy."""
    import numpy as np
    _, Xt, yt = inputs.holdout(wl.name, n_test, n=wl.N)
    Xq = torch.from_numpy(Xt).cuda()
    s = gabp.GabpSVM(**params)
    s.solve(X, y)
    plan = s.plan()
    f = s.predict(Xq)
    torch.cuda.synchronize()
    walls, kms = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        f = s.predict(Xq)
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        kms.append(s.timings()["predict_kernel_ms"])
    s.close()
    fh = f.cpu().numpy()
    acc = float(np.mean(np.where(fh >= 0, 1.0, -1.0) == yt))
    wall = float(np.median(walls))
    kms_med = float(np.median(kms))
    pairs = float(wl.N) * n_test
    # augmented rows (m + 2 <= 64): 32 or 64 columns, the solve's BF16 split
    # (three terms for FP32 handles)
    aug = wl.m + 2 <= 64
    m_pad = (32 if wl.m + 2 <= 32 else 64) if aug else (wl.m + 15) // 16 * 16
    # plan gram (gabp_gram): 0 = FP32 Gram (FP32 precision), 1..3 = BF16 split kinds
    gram = {0: "f32", 1: "bf16", 2: "bf16x3", 3: "bf16x6"}[plan["gram"]]
    if aug and gram == "f32":
        gram = "bf16x6"
    products = {"bf16": 1, "bf16x3": 3, "bf16x6": 6, "f32": 1}[gram]
    alg_flops = 2.0 * wl.m * pairs                  # the Gram dot products
    issued = 2.0 * m_pad * products * pairs         # MFMA work as issued (padding, split products)
    mfma_peak = MFMA_PEAK_TFLOPS["f32" if gram == "f32" else "bf16"]
    slots = PREDICT_SLOTS_PER_PAIR
    print(f"[bench] predict: {n_test} queries in {wall * 1e3:.2f} ms (kernel {kms_med:.2f} ms), "
          f"held-out accuracy {acc:.4f}", file=sys.stderr, flush=True)
    return {"queries": n_test, "train_N": wl.N, "gram": gram, "predictions_per_s": n_test / wall,
            "call_ms": wall * 1e3, "kernel_ms": kms_med, "held_out_accuracy": acc,
            "kernel": "k_predict_aug" if aug else "k_predict_mfma",
            # the binding unit is the MFMA pipe as the kernel issues it: the
            # split products over the padded (augmented) columns; the Gram's
            # algorithmic flops (2 m per pair) are reported beside it
            "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": mfma_peak,
                         "achieved": issued / (kms_med * 1e-3) / 1e12,
                         "frac": issued / (kms_med * 1e-3) / 1e12 / mfma_peak,
                         "issued_mfma_flops_per_pair": 2.0 * m_pad * products, "m_pad": m_pad,
                         "split_products": products, "alg_flops_per_pair": 2.0 * wl.m,
                         "alg_achieved": alg_flops / (kms_med * 1e-3) / 1e12,
                         "alg_frac": alg_flops / (kms_med * 1e-3) / 1e12 / mfma_peak,
                         "valu_slots_per_pair": slots,
                         "valu_frac": slots * pairs / (kms_med * 1e-3) / 1e9 / VALU_PEAK_GSLOT}}


def sparse_bench(torch, gabp, inputs, n, tau, steps=2, warmup=1):
    """Sparsified kernel at millions of points: the large workload's recipe
    (six unit clusters in 20 dimensions, gamma 0.05, MIXED) at N = n, pairs
    kept where exp(-gamma d^2) >= tau."""
    import numpy as np
    wl = inputs.make_workload("large", n=n)
    X = torch.from_numpy(wl.X).cuda()
    y = torch.from_numpy(wl.y).cuda()
    params = dict(kernel="rbf_sparse", sparse_tau=tau, gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam,
                  diag_delta=wl.delta, precision="mixed", tol_rel=wl.tol_rel, time_sweeps=1)
    wall, sweeps, ktime, klaunch, info = solve_steps(torch, gabp, wl, X, y, params, steps, warmup)
    plan, tm = info["plan"], info["timings"]
    E = plan["n_edges"]
    avg = ktime / max(klaunch, 1)
    ach = plan["alg_bytes_per_sweep"] / (avg * 1e-3) / 1e9 if klaunch else None
    print(f"[bench] sparse: N={n} edges={E} {sweeps} sweeps in {wall:.3f} s", file=sys.stderr, flush=True)
    return {"workload": f"large-like N={n} m={wl.m} gamma={wl.gamma:g}, kernel threshold {tau:g}, MIXED",
            "edges": E, "mean_degree": 2.0 * E / n, "sweeps_per_s": sweeps / wall, "solves_per_s": steps / wall,
            "sweeps_per_solve": info["sweeps_per_solve"], "reason": info["reason"],
            "graph_build_ms": tm["kbuild_ms"], "sweep_loop_ms": tm["sweep_loop_ms"],
            "roofline": {"bound": "hbm", "kernel": "k_sp_sweep + k_sp_gather", "achieved": ach,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS if ach else None,
                         "avg_launch_ms": avg, "alg_bytes_per_edge": plan["alg_bytes_per_pair"],
                         "alg_bytes_per_launch": plan["alg_bytes_per_sweep"]}}


def cpu_baseline(wl, adiag, depth, seconds):
    """The FP64 C oracle's stateless sweep (unroll depth `depth`, every kernel
    row rebuilt from the features) on the real N-point system, timed on a
    bounded sample of target rows: each sampled row forms its new aggregates
    from all N - 1 incoming messages, which is a sweep's per-node work at the
    full N, so rows/s / N is the oracle's sweep rate.  The aggregate history
    is the sweep-0 aggregates at every level (a sweep past the first `depth`
    sweeps unrolls every level; the work per pair does not depend on the
    values).  Timed at all host threads and at one."""
    import numpy as np

    from oracle import oracle_c
    oracle_c.build()
    N = wl.N
    T = depth + 1
    hP = np.tile(np.asarray(adiag, dtype=np.float64), (T, 1))
    hS = np.ones((T, N))
    nthr = oracle_c.max_threads()
    rng = np.random.default_rng(0)
    out = {}
    for threads in (nthr, 1):
        oracle_c.set_threads(threads)
        probe = np.sort(rng.choice(N, size=max(2 * threads, 8), replace=False))
        r = oracle_c.stateless_rows(wl.X, wl.y, wl.gamma, wl.lam, adiag, hP, hS, T, depth, probe)
        per_row = r["seconds"] / len(probe)
        n = int(min(N, max(len(probe), seconds / max(per_row, 1e-9))))
        rows = np.sort(rng.choice(N, size=n, replace=False))
        r = oracle_c.stateless_rows(wl.X, wl.y, wl.gamma, wl.lam, adiag, hP, hS, T, depth, rows)
        out[threads] = {"sweeps_per_s": n / r["seconds"] / N, "rows": n, "seconds": r["seconds"],
                        "pairs_per_s": n * (N - 1) / r["seconds"]}
        print(f"[bench] cpu oracle, {threads} threads: {n} rows in {r['seconds']:.2f} s", file=sys.stderr, flush=True)
    oracle_c.set_threads(nthr)
    return {"value": out[nthr]["sweeps_per_s"], "unit": "sweeps/s", "cores": nthr, "kind": "oracle",
            "value_1_thread": out[1]["sweeps_per_s"], "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "sample": (f"FP64 stateless sweep of the C oracle (depth {depth}, K' rebuilt from the features) on the "
                       f"full N={N} system: {out[nthr]['rows']} target rows with all {nthr} threads in "
                       f"{out[nthr]['seconds']:.1f} s, {out[1]['rows']} rows with 1 thread in "
                       f"{out[1]['seconds']:.1f} s, each row over all {N - 1} sources; sweeps/s = rows/s / N"),
            "threads": {str(k): v for k, v in out.items()}}


def cpu_full_solve(wl):
    """The C oracle's full FP64 solve (stored messages, Algorithm 2) of a
    small workload at all threads and at one: solves/s and sweeps/s."""
    from oracle import oracle_c
    nthr = oracle_c.max_threads()
    out = {}
    for threads in (nthr, 1):
        oracle_c.set_threads(threads)
        r = oracle_c.svm_solve(wl.X, wl.y, wl.gamma, wl.C, wl.lam, delta=wl.delta, tol_abs=wl.tol_abs,
                               tol_rel=wl.tol_rel)
        t = r["build_s"] + r["sweep_s"]
        out[str(threads)] = {"solves_per_s": 1.0 / t, "sweeps_per_s": r["sweeps"] / r["sweep_s"],
                             "sweeps": r["sweeps"], "status": r["status"]}
    oracle_c.set_threads(nthr)
    return out


def hbm_roof(plan, avg_ms, klaunch, kernel, traffic):
    achieved = plan["alg_bytes_per_sweep"] / (avg_ms * 1e-3) / 1e9 if klaunch else None
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "traffic_unit": "GB/launch", "kernel": kernel, "avg_launch_ms": avg_ms, "launches": klaunch,
            "alg_bytes_per_pair": plan["alg_bytes_per_pair"], "alg_bytes_per_launch": plan["alg_bytes_per_sweep"]}


def kernel_base_name(name):
    """A profiler's kernel name without the return type it may print first."""
    return name[5:] if name.startswith("void ") else name


def ingest_counters(fetch_dir, write_dir, calib_bytes, out_path):
    """Per-kernel HBM bytes per working launch from two rocprofv3 --pmc runs
    of this benchmark (FETCH_SIZE, then WRITE_SIZE; CSV output), each scaled
    by what the counter reads for the benchmark's calibration copy of
    `calib_bytes` bytes.  Launches that return at once after the stop rule
    (under 5% of the kernel's largest count) are left out."""
    import csv
    import glob

    def load(d, counter):
        rows = {}
        for fn in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(fn)):
                if r.get("Counter_Name") != counter:
                    continue
                rows.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return rows

    fetch, write = load(fetch_dir, "FETCH_SIZE"), load(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k]
    if not copy:
        raise SystemExit("no calibration copy in the counter runs (run the benchmark with --calib-copy-gb)")
    cf = max(fetch[copy[0]])
    cw = max(write[copy[0]])
    ff, wf = calib_bytes / (cf * 1024.0), calib_bytes / (cw * 1024.0)
    entries = {}
    for k in fetch:
        # this library's kernels only (library sorts and torch fills aside)
        if k not in write or not kernel_base_name(k).startswith("gabp::"):
            continue
        fv = [v for v in fetch[k] if v >= 0.05 * max(fetch[k])]
        wv = [v for v in write[k] if v >= 0.05 * max(write[k])] or write[k]
        fk, wk = sum(fv) / len(fv), sum(wv) / len(wv)
        entries[k] = {"fetch_kib": fk, "write_kib": wk, "fetch_bytes": fk * 1024 * ff, "write_bytes": wk * 1024 * wf,
                      "traffic_bytes": fk * 1024 * ff + wk * 1024 * wf, "launches": [len(fv), len(wv)]}
    out = {"kernel_source_sha256": device_source_hash(),
           "calibration": {"copy_bytes": calib_bytes, "fetch_factor": ff, "write_factor": wf,
                           "copy_fetch_kib": cf, "copy_write_kib": cw,
                           "note": "torch device copy (__amd_rocclr_copyBuffer); factor = known bytes / "
                                   "(counter KiB * 1024)"},
           "entries": entries}
    json.dump(out, open(out_path, "w"), indent=1, sort_keys=True)
    print(f"wrote {out_path}: {len(entries)} kernels, fetch factor {ff:.4f}, write factor {wf:.4f}")


def counter_traffic_kernel(path, name_prefix):
    """Traffic (GB per working launch) of the kernel whose name starts with
    name_prefix, if the stored counters match the current sources."""
    try:
        tj = json.load(open(path))
        if device_source_hash() != tj["kernel_source_sha256"]:
            return None
        for k, e in tj["entries"].items():
            if kernel_base_name(k).startswith(name_prefix):
                return e["traffic_bytes"] / 1e9
    except Exception:
        return None
    return None


# kernel names of the measured sweeps (template arguments: storage, message,
# aggregate type, K' source, Gram kind, levels, first sweep, series terms;
# the chunked sweep: storage, message, aggregate type, Gram kind, levels,
# series terms, tiles per chunk side)
TYPES = {"mixed": "float, double, double", "fp32": "float, float, float", "fp64": "double, double, double"}


def sweep_label(plan, edge_name, extra=""):
    """Short description of the sweep kernel a plan runs over the K' plane."""
    if plan.get("tile_chunk", 1) > 1:
        return f"k_sweep_chunk ({edge_name}, 2 x 2 tile chunks, K' materialised{extra})"
    return f"k_sweep ({edge_name}, K' materialised{extra})"


def sweep_kernel_name(precision, plan):
    """rocprofv3's name of the synchronous sweep kernel a plan launches over
    the materialised K' (template arguments as above)."""
    if plan["edge_state"] == 1:   # stored pair records (sweeps after the first)
        return f"gabp::k_sweep<{TYPES[precision]}, 0, 0, 0, false, 0>"
    if plan.get("tile_chunk", 1) > 1:
        return (f"gabp::k_sweep_chunk<{TYPES[precision]}, 0, {plan['stateless_depth']}, "
                f"{int(plan['series_reciprocal'])}, {plan['tile_chunk']}>")
    return (f"gabp::k_sweep<{TYPES[precision]}, 0, 0, {plan['stateless_depth']}, false, "
            f"{int(plan['series_reciprocal'])}>")


def main():
    a = parse()
    if a.ingest_counters:
        ingest_counters(a.ingest_counters[0], a.ingest_counters[1], a.calib_copy_gb * 1e9 or 4e9, a.traffic_json)
        return
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (the solver has no multi-GPU path); got --gpus {a.gpus}",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0810_1648_amd import gabp, inputs

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if a.serve_only:
        res = serving_bench(gabp, inputs, a.serve_requests, a.serve_load, a.serve_precision, a.serve_schedule,
                            steps_per_poll=a.serve_steps_per_poll, groups=a.serve_groups)
        print(json.dumps({"metric": "served GaBP solves: p50/p99 latency", "value": res["throughput_solves_per_s"],
                          "unit": "solves/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
                          "serving": res}), flush=True)
        return
    wl = inputs.make_workload(a.workload, n=a.n)
    N, m = wl.N, wl.m
    X = torch.from_numpy(wl.X).to(dev)
    y = torch.from_numpy(wl.y).to(dev)
    ref = alpha_ref(wl.name, wl.X, wl.y) if a.n is None else None
    aref = ref["alpha"] if ref is not None else None
    torch.cuda.synchronize()
    print(f"[bench] workload {wl.name} N={N} m={m} precision={a.precision} gram={a.gram}", file=sys.stderr, flush=True)

    base = dict(gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam, diag_delta=wl.delta, tol_abs=wl.tol_abs,
                tol_rel=wl.tol_rel, kstore=a.kstore, edge_state=a.edge, time_sweeps=1)
    params = dict(base, precision=a.precision, gram=a.gram)
    wall, sweeps, ktime, klaunch, info = solve_steps(torch, gabp, wl, X, y, params, a.steps, a.warmup,
                                                     certificate=True)
    print(f"[bench] main: {sweeps} sweeps in {wall:.3f} s, reason {info['reason']}, plan {info['plan']}",
          file=sys.stderr, flush=True)
    side = max(1, min(a.side_steps, a.steps))

    plain = None
    if not a.no_plain and a.precision != "fp32":
        pw, ps, pk, pl, pinfo = solve_steps(torch, gabp, wl, X, y, dict(base, precision="fp32"),
                                            a.steps, a.warmup)
        plain = {"sweeps_per_s": ps / pw, "solves_per_s": a.steps / pw, "sweeps_per_solve": pinfo["sweeps_per_solve"],
                 "reason": pinfo["reason"], "sweep_kernel_ms_avg": pk / max(pl, 1),
                 "edge_state": {1: "stored", 2: "stateless"}.get(pinfo["plan"]["edge_state"]),
                 "stateless_depth": pinfo["plan"]["stateless_depth"],
                 "err_vs_oracle": rel_err(pinfo["alpha"], aref),
                 "rel_diff_alpha_vs_main": rel_err(pinfo["alpha"], info["alpha"])}
        print(f"[bench] plain fp32: {ps} sweeps in {pw:.3f} s", file=sys.stderr, flush=True)

    if a.calib_copy_gb > 0:
        nel = int(a.calib_copy_gb * 1e9 / 4)
        src = torch.empty(nel, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    plan = info["plan"]
    avg_ms = ktime / max(klaunch, 1)
    pairs = N * (N - 1) / 2.0
    stateless = plan["edge_state"] == gabp.EDGE["stateless"]
    recompute = plan["kstore"] == gabp.KSTORE["recompute"]
    edge_name = "stateless" if stateless else "stored"
    traffic = counter_traffic_kernel(a.traffic_json, sweep_kernel_name(a.precision, plan))
    if not recompute:
        # the sweep streams the K' plane (and, with stored records, the four
        # pair-record planes): HBM-bound on its algorithmic bytes
        roof = hbm_roof(plan, avg_ms, klaunch, sweep_label(plan, edge_name), traffic)
    else:
        roof = {"bound": "alu", "kernel": "k_sweep_rc (stateless, K' recomputed)", "traffic": None}
    if stateless:
        slots = stateless_slots_per_pair(plan["stateless_depth"], int(plan["series_reciprocal"]), a.precision)
        if recompute:
            slots += recompute_slots(plan)
        valu = slots * pairs / (avg_ms * 1e-3) / 1e9 if klaunch else None
        roof.update({"valu_slots_per_pair": slots, "valu_gslot_per_s": valu, "valu_peak_gslot_per_s": VALU_PEAK_GSLOT,
                     "valu_frac": (valu / VALU_PEAK_GSLOT) if valu else None,
                     "stateless_depth": plan["stateless_depth"], "series_reciprocal": int(plan["series_reciprocal"]),
                     "stateless_rho": plan["stateless_rho"]})
        if recompute:
            roof.update({"achieved": valu, "peak": VALU_PEAK_GSLOT, "unit": "Gslot/s",
                         "frac": (valu / VALU_PEAK_GSLOT) if valu else None,
                         "avg_launch_ms": avg_ms, "launches": klaunch})

    stored_cmp = None
    if stateless and not a.no_stored:
        sw_, ss_, sk_, sl_, sinfo = solve_steps(torch, gabp, wl, X, y, dict(params, edge_state="stored"),
                                                 side, min(a.warmup, 1))
        sp = sinfo["plan"]
        stored_cmp = {"sweeps_per_s": ss_ / sw_, "solves_per_s": side / sw_, "steps": side,
                      "sweeps_per_solve": sinfo["sweeps_per_solve"], "reason": sinfo["reason"],
                      "err_vs_oracle": rel_err(sinfo["alpha"], aref),
                      "rel_diff_alpha_vs_main": rel_err(sinfo["alpha"], info["alpha"]),
                      "roofline": hbm_roof(sp, sk_ / max(sl_, 1), sl_, "k_sweep (stored, K' materialised)",
                                           counter_traffic_kernel(a.traffic_json, sweep_kernel_name(a.precision, sp)))}
        print(f"[bench] stored state: {ss_} sweeps in {sw_:.3f} s", file=sys.stderr, flush=True)

    grouped = None
    if not a.no_grouped:
        gw, gsw, gk, gl, ginfo = solve_steps(torch, gabp, wl, X, y, dict(params, schedule="grouped"),
                                             a.steps, a.warmup)
        gp = ginfo["plan"]
        grouped = {"schedule": "grouped (block Gauss-Seidel)", "groups": gp["sched_groups"],
                   "sweeps_per_s": gsw / gw, "solves_per_s": a.steps / gw,
                   "sweeps_per_solve": ginfo["sweeps_per_solve"], "reason": ginfo["reason"],
                   "sweep_ms_avg": gk / max(gl, 1),
                   "edge_state": {1: "stored", 2: "stateless"}.get(gp["edge_state"]),
                   "stateless_depth": gp["stateless_depth"],
                   "err_vs_oracle": rel_err(ginfo["alpha"], aref),
                   "rel_diff_alpha_vs_main": rel_err(ginfo["alpha"], info["alpha"]),
                   "solve_speedup_vs_sync": (a.steps / gw) / (a.steps / wall)}
        print(f"[bench] grouped schedule: {gsw} sweeps in {gw:.3f} s ({gp['sched_groups']} groups)",
              file=sys.stderr, flush=True)
    del X, y

    letter = None
    if not a.no_letter and a.workload != "letter":
        wl1 = inputs.make_workload("letter")
        X1, y1 = torch.from_numpy(wl1.X).to(dev), torch.from_numpy(wl1.y).to(dev)
        r1 = alpha_ref("letter", wl1.X, wl1.y)
        p1 = dict(gamma=wl1.gamma, C=wl1.C, lambda_aug=wl1.lam, diag_delta=wl1.delta, tol_rel=wl1.tol_rel,
                  precision="fp32", kstore="materialise", time_sweeps=1)
        lw, ls, lk, ll, linfo = solve_steps(torch, gabp, wl1, X1, y1, p1, max(side, 3), 1, certificate=True)
        lp = linfo["plan"]
        ledge = "stateless" if lp["edge_state"] == gabp.EDGE["stateless"] else "stored"
        letter = {"workload": f"letter-like N={wl1.N} m={wl1.m} RBF gamma={wl1.gamma:g} C={wl1.C:g}, plain FP32, "
                              f"K' materialised", "sweeps_per_s": ls / lw, "solves_per_s": max(side, 3) / lw,
                  "sweeps_per_solve": linfo["sweeps_per_solve"], "reason": linfo["reason"], "edge_state": ledge,
                  "stateless_depth": lp["stateless_depth"], "err_vs_oracle": rel_err(linfo["alpha"], r1["alpha"] if r1 is not None else None),
                  "certificate": linfo["certificate"],
                  "roofline": hbm_roof(lp, lk / max(ll, 1), ll, sweep_label(lp, ledge, ", FP32"), None)}
        print(f"[bench] letter: {ls} sweeps in {lw:.3f} s", file=sys.stderr, flush=True)
        del X1, y1

    large = None
    if not a.no_large and a.workload != "large":
        wl4 = inputs.make_workload("large")
        X4, y4 = torch.from_numpy(wl4.X).to(dev), torch.from_numpy(wl4.y).to(dev)
        r4 = alpha_ref("large", wl4.X, wl4.y)
        p4 = dict(gamma=wl4.gamma, C=wl4.C, lambda_aug=wl4.lam, diag_delta=wl4.delta, tol_rel=wl4.tol_rel,
                  precision="mixed", kstore="recompute", edge_state="stateless", time_sweeps=1)
        gw4, gs4, gk4, gl4, ginfo4 = solve_steps(torch, gabp, wl4, X4, y4, p4, side, 1, certificate=True)
        g4 = ginfo4["plan"]
        pairs4 = wl4.N * (wl4.N - 1) / 2.0
        ms4 = gk4 / max(gl4, 1)
        slots4 = stateless_slots_per_pair(g4["stateless_depth"], int(g4["series_reciprocal"]), "mixed") + \
            recompute_slots(g4)
        v4 = slots4 * pairs4 / (ms4 * 1e-3) / 1e9 if gl4 else None
        mp4 = (wl4.m + 15) // 16 * 16
        mf4 = 2.0 * mp4 * 6 * pairs4 / (ms4 * 1e-3) / 1e12 if gl4 else None
        large = {"workload": f"large-like N={wl4.N} m={wl4.m} RBF gamma={wl4.gamma:g} C={wl4.C:g}, MIXED, K' "
                             f"recomputed per tile, stateless", "sweeps_per_s": gs4 / gw4, "solves_per_s": side / gw4,
                 "sweeps_per_solve": ginfo4["sweeps_per_solve"], "reason": ginfo4["reason"],
                 "stateless_depth": g4["stateless_depth"], "device_bytes": g4["device_bytes"],
                 "err_vs_oracle": rel_err(ginfo4["alpha"], r4["alpha"] if r4 is not None else None),
                 "certificate": ginfo4["certificate"],
                 "roofline": {"bound": "alu", "kernel": "k_sweep_rc (stateless, K' recomputed)", "achieved": v4,
                              "peak": VALU_PEAK_GSLOT, "unit": "Gslot/s", "frac": v4 / VALU_PEAK_GSLOT if v4 else None,
                              "valu_slots_per_pair": slots4, "avg_launch_ms": ms4, "launches": gl4,
                              "mfma_issued_tflops": mf4, "mfma_frac": mf4 / MFMA_PEAK_TFLOPS["bf16"] if mf4 else None,
                              "traffic": None}}
        print(f"[bench] large: {gs4} sweeps in {gw4:.3f} s", file=sys.stderr, flush=True)
        del X4, y4

    predict = None
    if not a.no_predict:
        Xp, yp = torch.from_numpy(wl.X).to(dev), torch.from_numpy(wl.y).to(dev)
        predict = predict_bench(torch, gabp, inputs, wl, Xp, yp, params, a.predict_n)
        del Xp, yp

    sparse = None
    if not a.no_sparse:
        sparse = sparse_bench(torch, gabp, inputs, a.sparse_n, a.sparse_tau)

    serving = None
    if not a.no_serve:
        serving = serving_bench(gabp, inputs, a.serve_requests, a.serve_load, a.serve_precision, a.serve_schedule,
                                steps_per_poll=a.serve_steps_per_poll, groups=a.serve_groups)
        other = "sync" if a.serve_schedule == "grouped" else "grouped"
        o = serving_bench(gabp, inputs, a.serve_requests, a.serve_load, a.serve_precision, other, seq_sample=0,
                          steps_per_poll=a.serve_steps_per_poll, groups=a.serve_groups)
        serving[f"{other}_schedule"] = {k: o[k] for k in ("capacity_solves_per_s", "offered_rate_per_s", "p50_ms",
                                                         "p99_ms", "throughput_solves_per_s", "mean_sweeps",
                                                         "plan_mix", "err_vs_oracle")}
        mixed_prec = "mixed" if a.serve_precision != "mixed" else "fp32"
        o2 = serving_bench(gabp, inputs, a.serve_requests, a.serve_load, mixed_prec, a.serve_schedule, seq_sample=0,
                           steps_per_poll=a.serve_steps_per_poll, groups=a.serve_groups)
        serving[f"{mixed_prec}_precision"] = {k: o2[k] for k in ("capacity_solves_per_s", "offered_rate_per_s",
                                                                "p50_ms", "p99_ms", "throughput_solves_per_s",
                                                                "mean_sweeps", "plan_mix", "err_vs_oracle")}

    cpu = None
    if not a.no_cpu_baseline:
        adiag = ref["adiag"] if (ref is not None and "adiag" in ref.files) else None
        if adiag is None:
            from oracle import oracle_c
            oracle_c.build()
            _, adiag = oracle_c.svm_matvec(wl.X, wl.y, wl.gamma, wl.C, wl.lam, np.zeros(N), delta=wl.delta,
                                           want_diag=True)
        cpu = cpu_baseline(wl, adiag, max(1, plan["stateless_depth"]), a.cpu_seconds)
        cpu["full_solve_tiny"] = cpu_full_solve(inputs.make_workload("tiny"))

    dtype = {"mixed": "bf16x6-gram/f32-msg/f64-agg", "fp32": "f32", "fp64": "f64"}[a.precision]
    if a.precision == "mixed" and a.gram != "auto":
        dtype = f"{a.gram}-gram/f32-msg/f64-agg"
    line = {
        "metric": "GaBP sweeps/s + solves/s at N=100k RBF vs plain FP32; p50/p99 solve latency",
        "value": sweeps / wall,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{wl.name}-like N={N} m={m} RBF gamma={wl.gamma:g} C={wl.C:g} "
                               f"delta={wl.delta:g} tol_rel={wl.tol_rel:g}",
                   "N": N, "m": m, "precision": a.precision, "gram": a.gram if a.precision == "mixed" else None,
                   "kstore": {1: "materialise", 2: "recompute"}.get(plan["kstore"], plan["kstore"]),
                   "edge_state": edge_name,
                   "stateless_depth": plan["stateless_depth"] if stateless else None, "tile": plan["tile"]},
        "solves_per_s": a.steps / wall,
        "sweeps_per_solve": info["sweeps_per_solve"],
        "stop_reason": info["reason"],
        "err_vs_oracle": rel_err(info["alpha"], aref),
        "err_note": "||alpha - alpha*||_inf / ||alpha*||_inf against the oracle's FP64 alpha* (conjugate gradients "
                    "on the matrix-free FP64 product, Varah-certified to 1e-10)",
        "certificate": info["certificate"],
        "phase_ms": {k: info["timings"][k] for k in ("stage_ms", "kbuild_ms", "diag_ms", "sweep_loop_ms", "d2h_ms")},
        "plain_fp32": plain,
        "stored_state": stored_cmp,
        "grouped_schedule": grouped,
        "letter_fp32": letter,
        "large_recompute": large,
        "serving": serving,
        "sparse": sparse,
        "predict": predict,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

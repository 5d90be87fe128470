#!/usr/bin/env python3
"""Benchmark of the GaBP SVM hot path on one MI355X.

A step is one full solve (staging, K' build, diagonal weighting, sweeps to
the stop rule, alpha download) of the covertype-shaped workload: N = 100k
points, m = 54 features (43 uniform + 11 one-hot), RBF gamma = 0.5, C = 1,
labels from a random RBF teacher with 5% flips, inputs resident in device
memory before the timed region.  The headline `value` is GaBP sweeps per
second over the whole timed job (all sweeps of all steps / wall time); the
same line carries solves/s, the plain-FP32 comparison, the roofline of the
sweep kernel and the timed CPU oracle.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
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
# 4) and + lambda^2 (1)
RECOMPUTE_SLOTS_PER_PAIR = 9
# decision function, VALU slots per (query, training point) pair: distance
# from the Gram (add, fma), clamp, scale, exp2 (a transcendental: 4 slots),
# conversion to FP64 and the FP64 accumulation
PREDICT_SLOTS_PER_PAIR = 10


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


def counter_traffic(path, key):
    """HBM bytes per launch from the calibrated FETCH_SIZE + WRITE_SIZE counter
    runs recorded in profiles/, in GB; None when absent or when the kernel
    source has changed since the counters were taken."""
    import hashlib
    try:
        tj = json.load(open(path))
        if device_source_hash() != tj["kernel_source_sha256"]:
            return None
        e = tj["entries"].get(key)
        return None if e is None else e["traffic_bytes"] / 1e9
    except Exception:
        return None


def stateless_slots_per_pair(levels, series, precision="mixed"):
    """Algorithmic VALU issue slots per pair of one stateless sweep with
    `levels` unrolled levels (both directions of the pair), counting a
    multiply-add as one slot (contracted, as the compiler emits it) and a
    transcendental as four.
    Series reciprocals (`series` = number of terms at the top level; MIXED
    computes these messages in FP32 from FP32 K', so no conversion): a^2
    (1); the lower levels carry G = P / (-a^2) and F = E / a: the deepest
    level is G = 1/P~, F = -S/P~ of its source (free), each middle level
    forms, per direction, a^2 u^2 (1), G = u - a^2 u^2 G_rev (1),
    a F_rev - S (1) and F (1): 8; the top level forms, per direction,
    e = -a^2 G_rev u (2), the series (1 or 2), the accumulation of P (1,
    fused), a G (1), a F_rev - S (1) and the accumulation of E (1, fused):
    14 or 16.  With one level the top level runs from zero reverse
    messages: 7.
    Exact reciprocals: per direction and level the cavity precision (1), the
    reciprocal (FP32: 4; FP64: 4 + two Newton steps of 2 FMAs = 8) and the
    messages (4; 3 at the top, where the accumulations fuse); MIXED adds the
    conversion of K' to FP64 (1)."""
    if series:
        if levels <= 1:
            return 7
        return 1 + 8 * (levels - 2) + 2 * (6 + int(series))
    cvt = 1 if precision == "mixed" else 0
    r_top = 4 if precision == "fp32" else 8
    r_low = 8 if precision == "fp64" else 4
    return cvt + 1 + 2 * (levels - 1) * (1 + r_low + 4) + 2 * (1 + r_top + 3)


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
    return ap.parse_args()


def solve_steps(torch, gabp, wl, X, y, params, steps, warmup):
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
        infos = [srv.result(t)[1] for t in tickets]
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
    m_pad = (wl.m + 15) // 16 * 16
    # plan gram (gabp_gram): 0 = FP32 Gram (FP32 precision), 1..3 = BF16 split kinds
    gram = {0: "f32", 1: "bf16", 2: "bf16x3", 3: "bf16x6"}[plan["gram"]]
    products = {"bf16": 1, "bf16x3": 3, "bf16x6": 6, "f32": 1}[gram]
    alg_flops = 2.0 * wl.m * pairs                  # the Gram dot products
    issued = 2.0 * m_pad * products * pairs         # MFMA work as issued (padding, split products)
    mfma_peak = MFMA_PEAK_TFLOPS["f32" if gram == "f32" else "bf16"]
    slots = PREDICT_SLOTS_PER_PAIR
    print(f"[bench] predict: {n_test} queries in {wall * 1e3:.2f} ms (kernel {kms_med:.2f} ms), "
          f"held-out accuracy {acc:.4f}", file=sys.stderr, flush=True)
    return {"queries": n_test, "train_N": wl.N, "gram": gram, "predictions_per_s": n_test / wall,
            "call_ms": wall * 1e3, "kernel_ms": kms_med, "held_out_accuracy": acc,
            "kernel": "k_predict_mfma",
            "roofline": {"bound": "mfma", "unit": "TFLOP/s", "peak": mfma_peak,
                         "achieved": alg_flops / (kms_med * 1e-3) / 1e12,
                         "frac": alg_flops / (kms_med * 1e-3) / 1e12 / mfma_peak,
                         "alg_flops_per_pair": 2.0 * wl.m, "issued_mfma_flops_per_pair": 2.0 * m_pad * products,
                         "issued_frac": issued / (kms_med * 1e-3) / 1e12 / mfma_peak,
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


def cpu_baseline(wl, n_full, sample_n):
    """Times the FP64 oracle's synchronous sweep on the first sample_n points
    of the same workload and scales its pair rate to N = n_full."""
    from oracle import oracle_c
    oracle_c.build()
    Xs, ys = wl.X[:sample_n], wl.y[:sample_n]
    nsw = 6
    r = oracle_c.time_sweeps(Xs, ys, wl.gamma, wl.C, 1.0 / n_full, nsw)
    pairs = sample_n * (sample_n - 1) / 2.0 * nsw
    rate = pairs / r["seconds"]
    return {"value": rate / (n_full * (n_full - 1) / 2.0), "unit": "sweeps/s", "cores": r["threads"],
            "kind": "oracle",
            "sample": f"{nsw} FP64 sweeps of the C oracle on the first {sample_n} points of the same "
                      f"workload ({r['seconds']:.1f} s); pair rate {rate:.3e}/s scaled to "
                      f"N={n_full} ({n_full * (n_full - 1) // 2} pairs per sweep)"}


def main():
    a = parse()
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
    torch.cuda.synchronize()
    print(f"[bench] workload {wl.name} N={N} m={m} precision={a.precision} gram={a.gram}", file=sys.stderr, flush=True)

    base = dict(gamma=wl.gamma, C=wl.C, lambda_aug=wl.lam, diag_delta=wl.delta, tol_abs=wl.tol_abs,
                tol_rel=wl.tol_rel, kstore=a.kstore, edge_state=a.edge, time_sweeps=1)
    params = dict(base, precision=a.precision, gram=a.gram)
    wall, sweeps, ktime, klaunch, info = solve_steps(torch, gabp, wl, X, y, params, a.steps, a.warmup)
    print(f"[bench] main: {sweeps} sweeps in {wall:.3f} s, reason {info['reason']}, plan {info['plan']}",
          file=sys.stderr, flush=True)

    plain = None
    if not a.no_plain and a.precision != "fp32":
        pw, ps, pk, pl, pinfo = solve_steps(torch, gabp, wl, X, y, dict(base, precision="fp32"),
                                            a.steps, a.warmup)
        diff = float(np.max(np.abs(pinfo["alpha"] - info["alpha"])) / np.max(np.abs(info["alpha"])))
        plain = {"sweeps_per_s": ps / pw, "solves_per_s": a.steps / pw, "sweeps_per_solve": pinfo["sweeps_per_solve"],
                 "reason": pinfo["reason"], "sweep_kernel_ms_avg": pk / max(pl, 1),
                 "edge_state": {1: "stored", 2: "stateless"}.get(pinfo["plan"]["edge_state"]),
                 "stateless_depth": pinfo["plan"]["stateless_depth"],
                 "rel_diff_alpha_vs_main": diff}
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
    traffic = counter_traffic(a.traffic_json, f"{wl.name}:{N}:{a.precision}:{plan['kstore']}:{plan['edge_state']}")
    recompute = plan["kstore"] == gabp.KSTORE["recompute"]
    if stateless:
        slots = stateless_slots_per_pair(plan["stateless_depth"], int(plan["series_reciprocal"]), a.precision)
        if recompute:
            slots += RECOMPUTE_SLOTS_PER_PAIR
        achieved = slots * pairs / (avg_ms * 1e-3) / 1e9 if klaunch else None
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_GSLOT, "unit": "Gslot/s",
                "frac": (achieved / VALU_PEAK_GSLOT) if achieved else None, "traffic": traffic,
                "traffic_unit": "GB/launch",
                "kernel": "k_sweep (stateless)", "avg_launch_ms": avg_ms, "launches": klaunch,
                "alg_slots_per_pair": slots, "stateless_depth": plan["stateless_depth"],
                "series_reciprocal": int(plan["series_reciprocal"]),
                "stateless_rho": plan["stateless_rho"],
                "hbm_alg_bytes_per_launch": plan["alg_bytes_per_sweep"],
                "hbm_frac": plan["alg_bytes_per_sweep"] / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if klaunch else None}
        if recompute and klaunch:
            # the Gram of every pair on MFMA, as issued (padded features, split products)
            gname = {1: "bf16", 2: "bf16x3", 3: "bf16x6"}.get(plan["gram"], "f32")
            products = {"bf16": 1, "bf16x3": 3, "bf16x6": 6, "f32": 1}[gname]
            m_pad = (m + 15) // 16 * 16
            mf = 2.0 * m_pad * products * pairs / (avg_ms * 1e-3) / 1e12
            roof.update({"kstore": "recompute", "recompute_slots_per_pair": RECOMPUTE_SLOTS_PER_PAIR,
                         "mfma_gram": gname, "mfma_issued_tflops": mf,
                         "mfma_frac": mf / MFMA_PEAK_TFLOPS["f32" if gname == "f32" else "bf16"]})
    else:
        achieved = plan["alg_bytes_per_sweep"] / (avg_ms * 1e-3) / 1e9 if klaunch else None
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
                "traffic_unit": "GB/launch",
                "kernel": "k_sweep (stored)", "avg_launch_ms": avg_ms, "launches": klaunch,
                "alg_bytes_per_launch": plan["alg_bytes_per_sweep"],
                "alg_bytes_per_pair": plan["alg_bytes_per_pair"]}

    stored_cmp = None
    if stateless and not a.no_stored:
        sw_, ss_, sk_, sl_, sinfo = solve_steps(torch, gabp, wl, X, y, dict(params, edge_state="stored"),
                                                 a.steps, a.warmup)
        sp = sinfo["plan"]
        s_ms = sk_ / max(sl_, 1)
        s_ach = sp["alg_bytes_per_sweep"] / (s_ms * 1e-3) / 1e9
        stored_cmp = {"sweeps_per_s": ss_ / sw_, "solves_per_s": a.steps / sw_,
                      "sweeps_per_solve": sinfo["sweeps_per_solve"], "reason": sinfo["reason"],
                      "rel_diff_alpha_vs_main": float(np.max(np.abs(sinfo["alpha"] - info["alpha"])) /
                                                      np.max(np.abs(info["alpha"]))),
                      "roofline": {"bound": "hbm", "achieved": s_ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": s_ach / HBM_PEAK_GBS, "kernel": "k_sweep (stored)",
                                   "traffic": counter_traffic(a.traffic_json, f"{wl.name}:{N}:{a.precision}:{sp['kstore']}:{sp['edge_state']}"),
                                   "traffic_unit": "GB/launch",
                                   "avg_launch_ms": s_ms, "launches": sl_,
                                   "alg_bytes_per_launch": sp["alg_bytes_per_sweep"],
                                   "alg_bytes_per_pair": sp["alg_bytes_per_pair"]}}
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
                   "rel_diff_alpha_vs_main": float(np.max(np.abs(ginfo["alpha"] - info["alpha"])) /
                                                   np.max(np.abs(info["alpha"]))),
                   "solve_speedup_vs_sync": (a.steps / gw) / (a.steps / wall)}
        print(f"[bench] grouped schedule: {gsw} sweeps in {gw:.3f} s ({gp['sched_groups']} groups)",
              file=sys.stderr, flush=True)

    predict = None
    if not a.no_predict:
        predict = predict_bench(torch, gabp, inputs, wl, X, y, params, a.predict_n)

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
                                                         "plan_mix")}

    cpu = None
    if not a.no_cpu_baseline:
        sn = a.cpu_sample_n or min(N, 20000)
        cpu = cpu_baseline(wl, N, sn)

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
        "dtype": {"mixed": "bf16-gram/f32-store/f64-math", "fp32": "f32", "fp64": "f64"}[a.precision],
        "data": "synthetic",
        "config": {"workload": f"{wl.name}-like N={N} m={m} RBF gamma={wl.gamma:g} C={wl.C:g} "
                               f"delta={wl.delta:g} tol_rel={wl.tol_rel:g}",
                   "N": N, "m": m, "precision": a.precision, "gram": a.gram if a.precision == "mixed" else None,
                   "kstore": {1: "materialise", 2: "recompute"}.get(plan["kstore"], plan["kstore"]),
                   "edge_state": {1: "stored", 2: "stateless"}.get(plan["edge_state"], plan["edge_state"]),
                   "stateless_depth": plan["stateless_depth"] if stateless else None, "tile": plan["tile"]},
        "solves_per_s": a.steps / wall,
        "sweeps_per_solve": info["sweeps_per_solve"],
        "stop_reason": info["reason"],
        "phase_ms": {k: info["timings"][k] for k in ("stage_ms", "kbuild_ms", "diag_ms", "sweep_loop_ms", "d2h_ms")},
        "plain_fp32": plain,
        "stored_state": stored_cmp,
        "serving": serving,
        "grouped_schedule": grouped,
        "sparse": sparse,
        "predict": predict,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

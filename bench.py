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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="covertype", choices=["covertype", "letter", "tiny", "large"])
    ap.add_argument("--n", type=int, default=None, help="override N (same recipe)")
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp32", "fp64"])
    ap.add_argument("--gram", default="auto", choices=["auto", "bf16", "bf16x3", "bf16x6"])
    ap.add_argument("--kstore", default="materialise", choices=["materialise", "recompute", "auto"])
    ap.add_argument("--edge", default="stored", choices=["stored", "stateless", "auto"])
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=0, help="oracle sample size (0 = auto)")
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
    print(f"[bench] main: {sweeps} sweeps in {wall:.3f} s, reason {info['reason']}", file=sys.stderr, flush=True)

    plain = None
    if not a.no_plain and a.precision != "fp32":
        pw, ps, pk, pl, pinfo = solve_steps(torch, gabp, wl, X, y, dict(base, precision="fp32"),
                                            a.steps, a.warmup)
        diff = float(np.max(np.abs(pinfo["alpha"] - info["alpha"])) / np.max(np.abs(info["alpha"])))
        plain = {"sweeps_per_s": ps / pw, "solves_per_s": a.steps / pw, "sweeps_per_solve": pinfo["sweeps_per_solve"],
                 "reason": pinfo["reason"], "sweep_kernel_ms_avg": pk / max(pl, 1),
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
    achieved = plan["alg_bytes_per_sweep"] / (avg_ms * 1e-3) / 1e9 if klaunch else None
    traffic = None
    if os.path.exists(a.traffic_json):
        try:
            tj = json.load(open(a.traffic_json))
            key = f"{wl.name}:{N}:{a.precision}:{a.kstore}:{a.edge}"
            traffic = tj.get(key)
        except Exception:
            traffic = None
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": traffic,
            "kernel": "k_sweep_stored", "avg_launch_ms": avg_ms, "launches": klaunch,
            "alg_bytes_per_launch": plan["alg_bytes_per_sweep"],
            "alg_bytes_per_pair": plan["alg_bytes_per_pair"]}

    cpu = None
    if not a.no_cpu_baseline:
        sn = a.cpu_sample_n or min(N, 20000)
        cpu = cpu_baseline(wl, N, sn)

    line = {
        "metric": "GaBP sweeps/s (+ solves/s) at N=100k RBF, mixed vs plain FP32",
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
                   "kstore": plan["kstore"], "edge_state": plan["edge_state"], "tile": plan["tile"]},
        "solves_per_s": a.steps / wall,
        "sweeps_per_solve": info["sweeps_per_solve"],
        "stop_reason": info["reason"],
        "phase_ms": {k: info["timings"][k] for k in ("stage_ms", "kbuild_ms", "diag_ms", "sweep_loop_ms", "d2h_ms")},
        "plain_fp32": plain,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Gaussian-KDE hot path on one MI355X.

Workload: n = 100,000 data points and m = 100,000 queries in d = 64 drawn
from a 20-component isotropic Gaussian mixture (means U[-5,5]^64, sigma
U[0.5,2]), a = 0.01.  One step runs the whole hot path over that input:
exact kernel density of all m queries (prep, matrix-core tile, reduction).

Prints one JSON line: Gaussian kernel evaluations per second (n*m per step
at a measured max relative error <= 1e-5 vs the FP64 oracle), the roofline
of the dominant kernel from per-launch HIP events, and the FP64 CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAKS = {"fp32": ("mfma", 157.3e12), "fp16_split": ("mfma", 2.5e15), "bf16_split": ("mfma", 2.5e15),
         "bf16_split3": ("mfma", 2.5e15)}
PRODUCTS = {"fp32": 1, "fp16_split": 3, "bf16_split": 3, "bf16_split3": 6}
TILE_KERNEL = {"fp32": "kde_tile_f32", "fp16_split": "kde_tile_fp16x3", "bf16_split": "kde_tile_bf16x3",
               "bf16_split3": "kde_tile_bf16x6"}


def parse_timing(txt: str) -> dict:
    out = {}
    for line in txt.strip().splitlines():
        name, cnt, tot = line.split()
        out[name] = (int(cnt), float(tot))
    return out


def cpu_baseline(X, Q, a, budget_s: float):
    import oracle
    threads = os.cpu_count() or 1
    done, t_total, chunk = 0, 0.0, 256
    while t_total < budget_s and done < Q.shape[0]:
        t0 = time.perf_counter()
        oracle.kde_exact(X, Q[done:done + chunk], a, nthreads=threads)
        t_total += time.perf_counter() - t0
        done += min(chunk, Q.shape[0] - done)
    return {"value": X.shape[0] * done / t_total, "unit": "Gaussian kernel evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{done} of the {Q.shape[0]} queries against all {X.shape[0]} points (FP64 direct differences,"
                      f" OpenMP over queries), {t_total:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="fp16_split", choices=sorted(PEAKS))
    ap.add_argument("--a", type=float, default=0.01)
    ap.add_argument("--check-queries", type=int, default=256)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (how the path would shard over "
              "several GPUs is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import numpy as np
    import torch

    import paper_2407_07096_amd as stag
    import synth

    lib = stag.load()
    lib.stag_timing_enable.argtypes = [ctypes.c_int32]
    lib.stag_timing_report.restype = ctypes.c_size_t
    lib.stag_timing_report.argtypes = [ctypes.c_char_p, ctypes.c_size_t]
    dev = torch.device("cuda:0")
    X, Q, info = synth.config_points(2)
    n, d, m = info["n"], info["d"], info["m"]
    Xd = torch.from_numpy(X).to(dev)
    Qd = torch.from_numpy(Q).to(dev)
    S = torch.empty(m, dtype=torch.float64, device=dev)

    def step():
        stag.kde_exact(Xd, Qd, args.a, form=args.form, S_out=S)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    buf = ctypes.create_string_buffer(1 << 16)
    lib.stag_timing_report(buf, len(buf))  # drop warmup records
    lib.stag_timing_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.stag_timing_enable(0)
    lib.stag_timing_report(buf, len(buf))
    timing = parse_timing(buf.value.decode())
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    evals = float(n) * m
    value = evals / (ms_per_step / 1e3)

    # accuracy of this run's result on sampled queries against the FP64 oracle
    import oracle
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(m, size=args.check_queries, replace=False))
    ref = oracle.kde_exact(X, Q[idx], args.a)
    got = S.cpu().numpy()[idx]
    max_rel = float(np.max(np.abs(got - ref) / ref))

    tk = TILE_KERNEL[args.form]
    cnt, tot = timing.get(tk, (0, float("nan")))
    avg_ms = tot / max(cnt, 1)
    bound, peak = PEAKS[args.form]
    flops = 2.0 * d * evals * PRODUCTS[args.form]
    achieved = flops / (avg_ms / 1e3)
    result = {
        "metric": "Gaussian kernel evals/sec at <=1e-5 rel err vs FP64; p50/p99 KDE query latency",
        "value": value,
        "unit": "Gaussian kernel evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16_split": "f16x3 (f32 accumulate, f64 sum)",
                  "bf16_split": "bf16x3 (f32 accumulate, f64 sum)",
                  "bf16_split3": "bf16x6 (f32 accumulate, f64 sum)"}[args.form],
        "data": "synthetic",
        "config": {"workload": "exact Gaussian KDE, n=100000 data, m=100000 queries, d=64, 20-component mixture "
                               "(sigma U[0.5,2]), a=%g" % args.a, "form": args.form, "n": n, "m": m, "d": d},
        "max_rel_err_sampled": max_rel,
        "checked_queries": int(args.check_queries),
        "kernels_ms_per_step": {k: v[1] / max(v[0], 1) * (v[0] / args.steps) for k, v in timing.items()},
        "roofline": {"kernel": tk, "bound": bound, "achieved": achieved / 1e12, "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "flops_per_launch": flops, "avg_launch_ms": avg_ms},
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(X, Q, args.a, args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark of the Gaussian-KDE hot path on one MI355X.

Headline (the timed steps): exact kernel density at the largest workload
that fits one GPU, n = 2,000,000 data points and m = 200,000 queries in
d = 128 drawn from a 50-component isotropic Gaussian mixture (means
U[-5,5]^128, sigma U[0.5,2]), a = 0.01 (seeded, synthetic; it stands in for
the large data sets of the paper's KDE comparison).  One step is one call of
the exact KDE (operand prep, matrix-core tiles in the fp16 hi+lo split form,
chunk reduction, underflow check) over all m queries, inputs resident in
HBM.  value = n*m Gaussian kernel evaluations per second of the step, quoted
at the relative error measured against the FP64 oracle on 1,000 sampled
queries (<= 1e-5).

After the timed steps, each in its own JSON object: the other arithmetic
forms on the same workload (error and tile time), the full hot-path step at
n = m = 100,000, d = 64 (exact KDE + CKNS index build and query + edge
sampling, each leg timed alone), the CKNS estimator at the paper-derived
default parameters, edge sampling of the 784-dimensional sparse workload in
exact and CKNS mode, the other kernels, random sampling, spectral clustering,
the KDE-tree sampler, the E2LSH table, a serving run (p50/p99) and the FP64
CPU oracle timed on a bounded sample of the headline workload.  One JSON line
is printed.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MFMA_PEAK = {"fp32": 157.3e12, "fp16_split": 2.5e15, "bf16_split": 2.5e15, "bf16_split3": 2.5e15,
             "fp16_centred": 2.5e15, "fp16_adaptive": 2.5e15}
PRODUCTS = {"fp32": 1, "fp16_split": 3, "bf16_split": 3, "bf16_split3": 6, "fp16_centred": 1, "fp16_adaptive": 1}
TILE_KERNEL = {"fp32": "kde_tile_f32c", "fp16_split": "kde_tile_fp16x3", "bf16_split": "kde_tile_bf16x3",
               "bf16_split3": "kde_tile_bf16x6", "fp16_centred": "kde_tile_fp16c", "fp16_adaptive": "kde_tile_fp16c"}
DTYPE = {"fp32": "f32", "fp16_split": "f16x3->f32->f64", "bf16_split": "bf16x3->f32->f64",
         "bf16_split3": "bf16x6->f32->f64", "fp16_centred": "f16->f32->f64",
         "fp16_adaptive": "f16 (f16x3 where selected)->f32->f64"}
# the form of the hot-path step, the edge sampler and the other d = 64 legs
STEP_FORM = "fp16_split"
# CKNS parameters of the 784-dimensional edge sampling
C4_LSH = dict(k1=1, k2_constant=8, p_offset=3)
HBM_PEAK = 8.0e12
FP64_PEAK = 78.6e12
FP32_PEAK = 157.3e12  # vector fp32 (published)
# CKNS parameters of the hot-path step's lsh leg: the cheapest setting found on
# that workload whose average relative error is below 0.1 (the acceptance
# level of the paper's KDE comparison), eps = 0.5
LSH = dict(eps=0.5, k1=1, k2_constant=8, p_offset=1, lsh_seed=3002)
HEADLINE_A = 0.01


def parse_timing(txt: str) -> dict:
    out = {}
    for line in txt.strip().splitlines():
        name, cnt, tot = line.split()
        out[name] = (int(cnt), float(tot))
    return out


class Timers:
    """The library's per-launch HIP event timers (stag_timing_*) around a
    region: per kernel name (launches, total ms)."""

    def __init__(self, lib, buf, torch):
        self.lib, self.buf, self.torch = lib, buf, torch

    def __enter__(self):
        self.torch.cuda.synchronize()
        self.lib.stag_timing_report(self.buf, len(self.buf))  # drop older records
        self.lib.stag_timing_enable(1)
        self.t0 = time.perf_counter()
        return self

    def __exit__(self, *exc):
        self.torch.cuda.synchronize()
        self.wall_s = time.perf_counter() - self.t0
        self.lib.stag_timing_enable(0)
        self.lib.stag_timing_report(self.buf, len(self.buf))
        self.t = parse_timing(self.buf.value.decode())
        return False


def cpu_baseline(X, Q, a, budget_s: float):
    import oracle
    threads = os.cpu_count() or 1
    done, t_total, chunk = 0, 0.0, 64
    while t_total < budget_s and done < Q.shape[0]:
        t0 = time.perf_counter()
        oracle.kde_exact(X, Q[done:done + chunk], a, nthreads=threads)
        t_total += time.perf_counter() - t0
        done += min(chunk, Q.shape[0] - done)
    # single-thread figure on a short sample
    done1, t1 = 0, 0.0
    while t1 < min(3.0, budget_s / 4) and done1 < Q.shape[0]:
        t0 = time.perf_counter()
        oracle.kde_exact(X, Q[done1:done1 + 1], a, nthreads=1)
        t1 += time.perf_counter() - t0
        done1 += 1
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), cpu)
    except OSError:
        pass
    return {"value": X.shape[0] * done / t_total, "unit": "Gaussian kernel evals/s", "cores": threads,
            "cpu_model": cpu, "kind": "oracle", "value_1thread": X.shape[0] * done1 / t1,
            "sample": f"{done} of the {Q.shape[0]} headline queries against all {X.shape[0]} points (d = "
                      f"{X.shape[1]}), exact FP64 direct differences with compensated log-sum-exp, OpenMP over "
                      f"queries; {t_total:.1f} s; one-thread figure from {done1} queries"}


def oracle_reference(X, Q, idx, a):
    import oracle
    return oracle.kde_exact(X, Q[idx], a)


def second_bandwidth_run(stag, torch, lib, buf, X, Q, Xd, Qd, idx, form: str, a: float, reps: int = 2):
    """The headline call at the workload's second bandwidth (a = 0.001):
    time per call and error against the FP64 oracle on the same sampled
    queries."""
    import numpy as np
    n, m = X.shape[0], Q.shape[0]
    S, B = stag.kde_exact(Xd, Qd, a, form=form, return_bound=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        stag.kde_exact(Xd, Qd, a, form=form, S_out=S)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    ref = oracle_reference(X, Q, idx, a)
    err = np.abs(S.cpu().numpy()[idx] - ref) / ref
    return {"workload": f"exact Gaussian KDE, n={n}, m={m}, d={X.shape[1]}, a={a}, form {form}", "ms": ms,
            "evals_per_s": float(n) * m / (ms / 1e3), "max_rel_err_sampled": float(err.max()),
            "max_bound_sampled": float(B.cpu().numpy()[idx].max()), "checked_queries": int(len(idx))}


def lsh_headline_run(stag, torch, lib, buf, Xd, Qd, a, idx, ref, exact_ms, reps: int = 2):
    """The CKNS estimator on the headline workload (n = 2e6, m = 2e5, d = 128):
    index build, query of all queries, candidates and accepted terms per
    query, and the error against the FP64 oracle on the headline's sampled
    queries, next to the exact call's query rate."""
    import numpy as np
    n, m = Xd.shape[0], Qd.shape[0]
    sel = torch.from_numpy(idx).to(Qd.device)
    out = {"workload": f"CKNS KDE over the headline workload (n={n}, m={m}, d={Xd.shape[1]}, a={a}), eps=0.5",
           "exact_queries_per_s": m / (exact_ms / 1e3), "settings": []}
    for kw in (dict(k1=1, k2_constant=8, p_offset=1), dict(k1=1, k2_constant=8, p_offset=0)):
        torch.cuda.synchronize()
        with Timers(lib, buf, torch) as tb:
            ix = stag.LshIndex(Xd, a, eps=0.5, seed=3003, **kw)
        S, st = ix.query(Qd[sel].contiguous(), stats=True)
        Sa = ix.query(Qd)  # warm-up of the full query
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ix.query(Qd)
        torch.cuda.synchronize()
        q_ms = (time.perf_counter() - t0) * 1e3 / reps
        with Timers(lib, buf, torch) as tq:
            ix.query(Qd)
        shape = dict(ix.shape)
        ix.close()
        err = np.abs(S.cpu().numpy() - ref) / ref
        out["settings"].append({
            "params": kw, "shape": shape, "build_ms": tb.wall_s * 1e3, "query_ms_all": q_ms,
            "queries_per_s": m / (q_ms / 1e3), "speedup_vs_exact": exact_ms / q_ms,
            "effective_evals_per_s": float(n) * m / (q_ms / 1e3),
            "kernel_evals_per_s": float(st["n_acc"].double().mean().item()) * m / (q_ms / 1e3),
            "candidates_per_query": float(st["n_cand"].double().mean().item()),
            "accepted_per_query": float(st["n_acc"].double().mean().item()),
            "avg_rel_err_sampled": float(err.mean()), "max_rel_err_sampled": float(err.max()),
            "frac_within_eps": float(np.mean(err <= 0.5)), "checked_queries": int(len(idx)),
            "query_kernels_ms": {k: v[1] for k, v in tq.t.items()}})
        del Sa
    return out


def forms_run(stag, torch, lib, buf, Xd, Qd, a, idx, ref, forms, n, m, d, reps: int = 2):
    """Exact KDE of the headline workload in other arithmetic forms: tile
    time, evaluations per second of the tile, matrix-core fraction (on the
    method's 2d flops per pair and on the hardware's products) and the error
    against the FP64 oracle on the headline's sampled queries next to the
    largest stated per-result bound."""
    import numpy as np
    S = torch.empty(m, dtype=torch.float64, device=Qd.device)
    B = torch.empty(m, dtype=torch.float64, device=Qd.device)
    out = {}
    for form in forms:
        stag.kde_exact(Xd, Qd, a, form=form, S_out=S)  # warm-up
        with Timers(lib, buf, torch) as tm:
            for _ in range(reps):
                stag.kde_exact(Xd, Qd, a, form=form, S_out=S, bound_out=B, return_bound=True)
        tk = TILE_KERNEL[form]
        tile_ms = tm.t[tk][1] / tm.t[tk][0]
        useful = 2.0 * d * n * m
        err = np.abs(S.cpu().numpy()[idx] - ref) / ref
        out[form] = {"call_ms": tm.wall_s * 1e3 / reps, "tile_ms": tile_ms,
                     "evals_per_s_call": n * m / (tm.wall_s / reps), "evals_per_s_tile": n * m / (tile_ms / 1e3),
                     "frac_of_peak_useful": useful / (tile_ms / 1e3) / MFMA_PEAK[form],
                     "frac_of_peak_hardware": useful * PRODUCTS[form] / (tile_ms / 1e3) / MFMA_PEAK[form],
                     "max_rel_err_sampled": float(err.max()), "max_bound_sampled": float(B.cpu().numpy()[idx].max()),
                     "meets_1e-5": bool(err.max() <= 1e-5)}
    return out

def hot_path_step_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, form: str, a: float, steps: int, n_check: int = 256):
    """The full hot path at n = m = 100,000, d = 64 (20-component mixture,
    a = 0.01): exact KDE of all queries, CKNS index build and query, exact
    edge sampling (17 draws per node).  Each leg is timed alone, then the
    whole step in order and with its legs on three streams."""
    import numpy as np

    import oracle
    n, d = X.shape
    m = Q.shape[0]
    S = torch.empty(m, dtype=torch.float64, device=dev)
    lsh_kw = {k: v for k, v in LSH.items() if k not in ("eps", "lsh_seed")}
    res = {}

    def exact_leg():
        stag.kde_exact(Xd, Qd, a, form=form, S_out=S)

    def lsh_leg():
        idx = stag.LshIndex(Xd, a, eps=LSH["eps"], seed=LSH["lsh_seed"], **lsh_kw)
        res["lsh"] = idx.query(Qd)
        idx.close()

    def graph_leg():
        res["graph"] = stag.simgraph_sample(Xd, a, mode="exact", form=form, seed=4002)

    def step():
        lsh_leg()
        exact_leg()
        graph_leg()

    legs = {}
    for name, fn in (("exact", exact_leg), ("lsh", lsh_leg), ("graph", graph_leg)):
        fn()
        with Timers(lib, buf, torch) as tm:
            for _ in range(steps):
                fn()
        legs[name] = {"ms": tm.wall_s * 1e3 / steps,
                      "kernels_ms": {k: v[1] / steps for k, v in tm.t.items()}}
    step()
    with Timers(lib, buf, torch) as tm:
        for _ in range(steps):
            step()
    ms_step = tm.wall_s * 1e3 / steps
    per_step = {k: v[1] / steps for k, v in tm.t.items()}
    timing = tm.t
    S_main = S.clone()
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(m, size=n_check, replace=False))
    ref = oracle.kde_exact(X, Q[idx], a)
    max_rel = float(np.max(np.abs(S_main.cpu().numpy()[idx] - ref) / ref))
    lsh_rel = float(np.mean(np.abs(res["lsh"].cpu().numpy()[idx] - ref) / ref))
    index = stag.LshIndex(Xd, a, eps=LSH["eps"], seed=LSH["lsh_seed"], **lsh_kw)
    _, st = index.query(Qd, stats=True)
    n_cand = int(st["n_cand"].sum().item())
    n_acc = int(st["n_acc"].sum().item())
    index.close()
    t_lsh = sum(v for k, v in per_step.items() if k.startswith("lsh_")) / 1e3
    evals = float(n) * m
    # rooflines of the step's kernels
    tk = TILE_KERNEL[form]
    roofs = {}
    c, tot = timing[tk]
    tile_avg = tot / c
    useful = 2.0 * d * evals
    roofs[tk] = {"bound": "mfma", "achieved": useful / (tile_avg / 1e3) / 1e12, "peak": MFMA_PEAK[form] / 1e12,
                 "unit": "TFLOP/s", "frac": useful / (tile_avg / 1e3) / MFMA_PEAK[form],
                 "frac_hardware": useful * PRODUCTS[form] / (tile_avg / 1e3) / MFMA_PEAK[form],
                 "avg_launch_ms": tile_avg, "launches_per_step": c / steps,
                 "algorithmic": f"2*d flops per pair x n*m = {useful:.3e} (x{PRODUCTS[form]} products on the "
                                f"matrix cores); the exact KDE and the edge sampler's self pass"}
    if "lsh_join" in timing:
        c, tot = timing["lsh_join"]
        fl = 3.0 * d * n_cand
        roofs["lsh_join"] = {"bound": "alu", "achieved": fl / (tot / c / 1e3) / 1e12, "peak": FP32_PEAK / 1e12,
                             "unit": "TFLOP/s", "frac": fl / (tot / c / 1e3) / FP32_PEAK, "avg_launch_ms": tot / c,
                             "algorithmic": f"{n_cand} (query, bucket member) pairs x 3d fp32 flops"}
    if "lsh_hash_queries" in timing:
        c, tot = timing["lsh_hash_queries"]
        sh = stag.lsh_derive(n, a, LSH["eps"], **lsh_kw)
        fl = 2.0 * d * m * sh["K1"] * sh["J"] * sh["L"] * sh["K"]
        roofs["lsh_hash_queries"] = {"bound": "alu", "achieved": fl / (tot / c / 1e3) / 1e12,
                                     "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s", "frac": fl / (tot / c / 1e3) / FP64_PEAK,
                                     "avg_launch_ms": tot / c, "algorithmic": "2*d fp64 flops per (query, projection)"}
    if "simgraph_draw_exact" in timing:
        c, tot = timing["simgraph_draw_exact"]
        s = stag.draws_per_node(n)
        by = n * s * (32 * 4 * d + 8 * 2 * ((n + 4095) // 4096) + 4 * 2 * 128)
        roofs["simgraph_draw_exact"] = {"bound": "hbm", "achieved": by / (tot / c / 1e3) / 1e9, "peak": 8000.0,
                                        "unit": "GB/s", "frac": by / (tot / c / 1e3) / HBM_PEAK,
                                        "avg_launch_ms": tot / c,
                                        "algorithmic": "per draw: the 32 rows of its tile (4d bytes each), its "
                                                       "row's chunk sums and one 128-tile group of tile sums"}
    # the same step with its legs on three streams (default priority)
    streams = [torch.cuda.Stream(device=dev) for _ in range(3)]
    S2 = torch.empty(m, dtype=torch.float64, device=dev)

    def step_overlapped():
        with torch.cuda.stream(streams[0]):
            stag.kde_exact(Xd, Qd, a, form=form, S_out=S2)
        with torch.cuda.stream(streams[1]):
            stag.simgraph_sample(Xd, a, mode="exact", form=form, seed=4002)
        with torch.cuda.stream(streams[2]):
            ix2 = stag.LshIndex(Xd, a, eps=LSH["eps"], seed=LSH["lsh_seed"], **lsh_kw)
            ix2.query(Qd)
            ix2.close()

    torch.cuda.synchronize()
    step_overlapped()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step_overlapped()
    torch.cuda.synchronize()
    ms_ov = (time.perf_counter() - t0) * 1e3 / steps
    src, dst, w, deg = (t.cpu().numpy() for t in res["graph"])
    out = {"workload": f"n={n} data, m={m} queries, d={d}, 20-component mixture (sigma U[0.5,2]), a={a}: exact KDE "
                       f"({form}) + CKNS LSH KDE (build+query, eps={LSH['eps']}, k1={LSH['k1']}, "
                       f"k2_constant={LSH['k2_constant']}, p_offset={LSH['p_offset']}) + exact edge sampling "
                       f"({stag.draws_per_node(n)} draws/node)",
           "steps": steps, "ms_per_step": ms_step, "evals_per_s": evals / (ms_step / 1e3),
           "legs_alone": legs, "exact_kde_ms": legs["exact"]["ms"],
           "exact_evals_per_s": evals / (legs["exact"]["ms"] / 1e3),
           "max_rel_err_sampled": max_rel, "checked_queries": n_check,
           "lsh_avg_rel_err_sampled": lsh_rel, "lsh_candidates_per_query": n_cand / m,
           "lsh_accepted_per_query": n_acc / m,
           "lsh_leg": {"kernel_ms_per_step": t_lsh * 1e3, "effective_evals_per_s": n * m / t_lsh,
                       "distance_evals_per_s": n_cand / t_lsh, "kernel_evals_per_s": n_acc / t_lsh},
           "graph_edges": int(src.size), "graph_valid_edges": int((dst >= 0).sum()),
           "kernels_ms_per_step": per_step, "rooflines": roofs,
           "overlapped_legs": {"ms_per_step": ms_ov, "exact_results_identical": bool(torch.equal(S2, S_main))}}
    return out, res["graph"]


def lsh_defaults_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, a: float, m_sub: int = 2000, n_check: int = 64):
    """The CKNS estimator at the paper-derived default parameters (eps = 0.5:
    K1 = ceil(log2(n)/eps^2), L = ceil(log2 n), K from the recovery target,
    J = ceil(log2 n) levels) over the hot-path step's data: index build, query
    of m_sub queries, work counts, and the average and largest relative error
    against the exact density."""
    import numpy as np

    import oracle
    n, d = X.shape
    rng = np.random.default_rng(2007)
    qi = np.sort(rng.choice(Q.shape[0], size=m_sub, replace=False))
    Qs = torch.from_numpy(np.ascontiguousarray(Q[qi])).to(dev)
    sh = stag.lsh_derive(n, a, 0.5)
    torch.cuda.synchronize()
    with Timers(lib, buf, torch) as tb:
        idx = stag.LshIndex(Xd, a, eps=0.5, seed=3002)
    build_ms = tb.wall_s * 1e3
    idx.query(Qs[:128])  # warm-up
    with Timers(lib, buf, torch) as tq:
        S, st = idx.query(Qs, stats=True)
    idx.close()
    ex = stag.kde_exact(Xd, Qs, a, form="fp16_split")
    Sh, exh = S.cpu().numpy(), ex.cpu().numpy()
    rel = np.abs(Sh - exh) / exh
    ref = oracle.kde_exact(X, Q[qi[:n_check]], a)
    return {"workload": f"CKNS KDE, default parameters (eps=0.5), n={n}, d={d}, a={a}; {m_sub} sampled queries",
            "shape": sh, "build_ms": build_ms, "build_kernels_ms": {k: v[1] for k, v in tb.t.items()},
            "query_ms": tq.wall_s * 1e3, "queries_per_s": m_sub / tq.wall_s,
            "query_kernels_ms": {k: v[1] for k, v in tq.t.items()},
            "candidates_per_query": float(st["n_cand"].double().mean().item()),
            "accepted_per_query": float(st["n_acc"].double().mean().item()),
            "avg_rel_err_vs_exact": float(rel.mean()), "max_rel_err_vs_exact": float(rel.max()),
            "frac_within_eps": float(np.mean(rel <= 0.5)),
            "exact_vs_oracle_max_rel_err": float(np.max(np.abs(exh[:n_check] - ref) / ref))}


def c4_run(stag, torch, dev, lib, buf, s_lsh: dict, n_nodes_law: int = 256):
    """Edge sampling of the 784-dimensional sparse workload (n = 70,000,
    entries 0 w.p. 0.8 else U[0,1], a = 1e-3, ceil(log2 n) = 17 draws per
    node) in exact mode (the wide fp32 tile, and the wide fp16 split tile) and
    CKNS mode.  Reported: times,
    draws/s, the CKNS-mode degree estimates against the exact degrees, and
    total-variation distances between histograms of the drawn edges' squared
    distances: CKNS mode vs exact mode, and each mode vs the exact law of
    n_nodes_law sampled nodes (the noise floor of the comparison)."""
    import numpy as np

    import synth
    n, d, a = 70_000, 784, 1e-3
    X = synth.sparse_uniform(n, d, 1004)
    Xd = torch.from_numpy(X).to(dev)
    out = {"workload": f"edge sampling n={n}, d={d} (80% zeros, else U[0,1]), a={a}, "
                       f"{stag.draws_per_node(n)} draws/node", "modes": {}}
    graphs = {}
    for key, mode, kw in (("exact", "exact", dict(form="fp32")),
                          ("exact_fp16_split", "exact", dict(form="fp16_split")),
                          ("lsh", "lsh", dict(eps=0.5, lsh_seed=3004, **s_lsh))):
        stag.simgraph_sample(Xd, a, mode=mode, seed=4004, **kw)  # warm-up
        with Timers(lib, buf, torch) as tm:
            g = stag.simgraph_sample(Xd, a, mode=mode, seed=4004, **kw)
        graphs[key] = g
        out["modes"][key] = {"ms": tm.wall_s * 1e3, "draws_per_s": n * stag.draws_per_node(n) / tm.wall_s,
                             "kernels_ms": {k: v[1] for k, v in tm.t.items()}}
    out["modes"]["lsh"]["params"] = dict(eps=0.5, **s_lsh)

    def drawn_d2(g):
        src, dst = g[0], g[1]
        ok = dst >= 0
        s_, d_ = src[ok], dst[ok]
        vals = []
        for c0 in range(0, s_.numel(), 100_000):
            xs, xd = Xd[s_[c0:c0 + 100_000]], Xd[d_[c0:c0 + 100_000]]
            vals.append(((xs.double() - xd.double()) ** 2).sum(1))
        return torch.cat(vals).cpu().numpy()

    de, dl, dh = drawn_d2(graphs["exact"]), drawn_d2(graphs["lsh"]), drawn_d2(graphs["exact_fp16_split"])
    rng = np.random.default_rng(4104)
    nodes = rng.choice(n, size=n_nodes_law, replace=False)
    lw, ld = [], []
    X64 = Xd.double()
    for i in nodes:
        dd = ((X64 - X64[int(i)]) ** 2).sum(1)
        row = torch.exp(-a * dd)
        row[int(i)] = 0.0
        lw.append((row / row.sum()).cpu().numpy())
        ld.append(dd.cpu().numpy())
    del X64
    lw, ld = np.concatenate(lw) / n_nodes_law, np.concatenate(ld)
    lo, hi = float(min(de.min(), dl.min())), float(max(de.max(), dl.max()))
    bins = np.linspace(lo, hi, 65)

    def hist(v, w=None):
        h, _ = np.histogram(np.clip(v, lo, hi), bins=bins, weights=w)
        return h / h.sum()

    he, hl, hh, hlaw = hist(de), hist(dl), hist(dh), hist(ld, lw)
    deg_e, deg_l = graphs["exact"][3].cpu().numpy(), graphs["lsh"][3].cpu().numpy()
    drel = np.abs(deg_l - deg_e) / deg_e
    out["tv_drawn_d2_lsh_vs_exact"] = float(0.5 * np.abs(hl - he).sum())
    out["tv_drawn_d2_exact_vs_law"] = float(0.5 * np.abs(he - hlaw).sum())
    out["tv_drawn_d2_lsh_vs_law"] = float(0.5 * np.abs(hl - hlaw).sum())
    out["tv_drawn_d2_exact_fp16_split_vs_law"] = float(0.5 * np.abs(hh - hlaw).sum())
    gs, gf = graphs["exact_fp16_split"], graphs["exact"]
    out["exact_fp16_split_vs_fp32"] = {
        "same_draws": float((gs[1] == gf[1]).double().mean().item()),
        "max_rel_degree_diff": float((torch.abs(gs[3] - gf[3]) / gf[3]).max().item())}
    out["lsh_degree_rel_err"] = {"median": float(np.median(drel)), "p90": float(np.quantile(drel, 0.9)),
                                 "max": float(drel.max())}
    out["histogram"] = f"64 bins of ||x_i - x_j||^2 over [{lo:.1f}, {hi:.1f}]; law from {n_nodes_law} nodes' exact rows"
    del Xd, graphs
    torch.cuda.empty_cache()
    return out

def kernels_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, form: str, n_check: int = 32):
    """Exact KDE with each kernel function of the paper (Gaussian a = 0.01,
    exponential and logistic a = 0.2) over the step's data and queries in one
    form: tile time, pairs/s, matrix-core fraction (the same products as the
    Gaussian tile) and the error against the FP64 oracle on sampled queries."""
    import numpy as np

    import oracle
    n, d = X.shape
    m = Q.shape[0]
    rng = np.random.default_rng(2005)
    idx = np.sort(rng.choice(m, size=n_check, replace=False))
    S = torch.empty(m, dtype=torch.float64, device=dev)
    B = torch.empty(m, dtype=torch.float64, device=dev)
    out = {"workload": f"exact KDE n={n}, m={m}, d={d}, form {form}", "checked_queries": n_check, "kernels": {}}
    for kernel, a in [("gaussian", 0.01), ("exponential", 0.2), ("logistic", 0.2)]:
        stag.kde_exact(Xd, Qd, a, form=form, S_out=S, kernel=kernel)  # warm-up
        torch.cuda.synchronize()
        lib.stag_timing_report(buf, len(buf))
        lib.stag_timing_enable(1)
        reps = 3
        for _ in range(reps):
            stag.kde_exact(Xd, Qd, a, form=form, S_out=S, bound_out=B, return_bound=True, kernel=kernel)
        torch.cuda.synchronize()
        lib.stag_timing_enable(0)
        lib.stag_timing_report(buf, len(buf))
        t = parse_timing(buf.value.decode())
        tk = TILE_KERNEL[form]
        tile_ms = t[tk][1] / t[tk][0]
        flops = 2.0 * d * n * m * PRODUCTS[form]
        ref = oracle.kde_kernel(X, Q[idx], a, kernel)
        err = np.abs(S.cpu().numpy()[idx] - ref) / ref
        out["kernels"][kernel] = {"a": a, "tile_ms": tile_ms, "pairs_per_s": n * m / (tile_ms / 1e3),
                                  "frac_of_peak": flops / (tile_ms / 1e3) / MFMA_PEAK[form],
                                  "max_rel_err_sampled": float(err.max()),
                                  "max_bound_sampled": float(B.cpu().numpy()[idx].max())}
    return out


def spectral_run(stag, torch, lib, buf, graph, n: int, k: int, labels_true, seed: int = 4003):
    """Spectral clustering of the step's sampled graph (k = the mixture's
    component count): embedding (bottom-k eigenvectors of the normalised
    Laplacian) and k-means times with their kernels, the largest eigen-residual
    ||N u - lambda u|| recomputed on the host from the downloaded graph, and
    the purity of the clusters against the mixture components."""
    import numpy as np
    from scipy.sparse import coo_matrix
    src, dst, w, _ = graph
    stag.spectral_embedding(n, src, dst, w, k, seed=seed)  # warm-up
    torch.cuda.synchronize()
    lib.stag_timing_report(buf, len(buf))
    lib.stag_timing_enable(1)
    t0 = time.perf_counter()
    lam, U, iters = stag.spectral_embedding(n, src, dst, w, k, seed=seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lab, _, rounds, _ = stag.kmeans(U, k, seed=seed)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lib.stag_timing_enable(0)
    lib.stag_timing_report(buf, len(buf))
    tm = parse_timing(buf.value.decode())
    s_, d_, w_ = (t.cpu().numpy() for t in (src, dst, w))
    ok = d_ >= 0
    A = coo_matrix((np.concatenate([w_[ok], w_[ok]]), (np.concatenate([s_[ok], d_[ok]]),
                                                       np.concatenate([d_[ok], s_[ok]]))), shape=(n, n)).tocsr()
    deg = np.asarray(A.sum(axis=1)).ravel()
    dinv = np.where(deg > 0, 1.0 / np.sqrt(np.where(deg > 0, deg, 1.0)), 0.0)
    Uh, lh = U.cpu().numpy(), lam.cpu().numpy()
    NU = Uh - dinv[:, None] * (A @ (dinv[:, None] * Uh))
    res = float(np.linalg.norm(NU - Uh * lh[None, :], axis=0).max())
    labh = lab.cpu().numpy()
    purity = sum(np.bincount(labh[labels_true == c]).max() for c in range(k) if np.any(labels_true == c)) / n
    return {"workload": f"spectral clustering of the step's sampled graph: n={n}, {int(ok.sum())} edges, k={k}",
            "embedding_ms": (t1 - t0) * 1e3, "kmeans_ms": (t2 - t1) * 1e3, "filter_steps": iters,
            "kmeans_rounds": rounds, "eigenvalues_head": [float(v) for v in lh[:4]],
            "eigenvalue_k": float(lh[-1]), "max_residual_host": res, "purity_vs_components": float(purity),
            "kernels_ms": {kk: v[1] for kk, v in tm.items()}}


def tree_run(stag, torch, lib, buf, X, Xd, a: float, graph, labels, k: int, s: int = 17, t: int = 32,
             t_deg: int = 1024, seed: int = 4004):
    """KDE-tree edge sampler (random-sampling node estimates, t per estimate,
    t_deg for the degrees) over the step's data: time and draws/s with its
    kernels, fp64 rate of the draw kernel against the vector fp64 peak, and
    against the step's exact sampler: the share of sampled weight inside the
    mixture components, the degree estimates' error, and the purity of
    spectral clustering on each graph; draws of 32 rows against the oracle."""
    import numpy as np

    import oracle
    n, d = X.shape
    stag.simgraph_sample_tree(Xd, a, s, t, t_deg, seed)  # warm-up
    torch.cuda.synchronize()
    lib.stag_timing_report(buf, len(buf))
    lib.stag_timing_enable(1)
    t0 = time.perf_counter()
    tg = stag.simgraph_sample_tree(Xd, a, s, t, t_deg, seed)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.stag_timing_enable(0)
    lib.stag_timing_report(buf, len(buf))
    tm = parse_timing(buf.value.decode())
    h = max(0, int(np.ceil(np.log2(-(-n // 32)))))
    values = n * s * (h * 2 * t + 32)  # kernel values per launch of the draw kernel (upper count)
    draw_ms = tm["tree_draws"][1]
    flops64 = values * 3.0 * d  # difference, product, sum per coordinate

    def stats(g):
        src, dst, w, deg = (x.cpu().numpy() for x in g)
        ok = dst >= 0
        inside = float(w[ok][labels[src[ok]] == labels[dst[ok]]].sum() / w[ok].sum())
        lam, U, _ = stag.spectral_embedding(n, g[0], g[1], g[2], k, seed=seed)
        lab, _, _, _ = stag.kmeans(U, k, seed=seed)
        labh = lab.cpu().numpy()
        purity = sum(np.bincount(labh[labels == c]).max() for c in range(k) if np.any(labels == c)) / n
        return inside, float(purity), deg

    in_tree, pur_tree, deg_tree = stats(tg)
    in_exact, pur_exact, deg_exact = stats(graph)
    drel = np.abs(deg_tree - deg_exact) / deg_exact
    lo, hi = n // 2, n // 2 + 32
    ref = oracle.simgraph_tree(X, a, s, t, t_deg, seed, rows=(lo, hi))
    dst_h = tg[1].cpu().numpy()[lo * s:hi * s]
    return {"workload": f"KDE-tree edge sampling n={n}, d={d}, a={a}, s={s}, t={t}, t_deg={t_deg}",
            "wall_ms": (t1 - t0) * 1e3, "draws_per_s": n * s / (t1 - t0),
            "kernels_ms": {kk: v[1] for kk, v in tm.items()},
            "draw_kernel_fp64_tflops": flops64 / (draw_ms / 1e3) / 1e12, "fp64_vector_peak_tflops": 78.6,
            "weight_share_inside_components": {"tree": in_tree, "exact": in_exact},
            "spectral_purity": {"tree": pur_tree, "exact": pur_exact},
            "degree_rel_err_vs_exact": {"median": float(np.median(drel)), "max": float(drel.max())},
            "oracle_draws_differing_of_32_rows": int(np.sum(dst_h != ref[1]))}


def rs_run(stag, torch, lib, buf, X, Q, Xd, Qd, a: float, form: str, n_check: int = 32):
    """Random-sampling KDE (the paper's sampling baseline) over the step's
    data and queries at s = n/100 and n/10 samples: time, throughput of
    estimated queries, error against the exact density of every query (GPU,
    fp32 form), and parity with the oracle's estimator on sampled queries."""
    import numpy as np

    import oracle
    n = X.shape[0]
    m = Q.shape[0]
    exact = stag.kde_exact(Xd, Qd, a, form="fp32").cpu().numpy()
    rng = np.random.default_rng(2006)
    idx = np.sort(rng.choice(m, size=n_check, replace=False))
    out = {"workload": f"random-sampling KDE over n={n}, m={m}, d={X.shape[1]}, a={a}, form {form}", "samples": {}}
    for s in (n // 100, n // 10):
        stag.kde_random_sample(Xd, Qd, a, s, seed=7, form=form)  # warm-up
        torch.cuda.synchronize()
        lib.stag_timing_report(buf, len(buf))
        lib.stag_timing_enable(1)
        t0 = time.perf_counter()
        S = stag.kde_random_sample(Xd, Qd, a, s, seed=7, form=form)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lib.stag_timing_enable(0)
        lib.stag_timing_report(buf, len(buf))
        tm = parse_timing(buf.value.decode())
        Sh = S.cpu().numpy()
        rel = np.abs(Sh - exact) / exact
        ref, _ = oracle.kde_random_sample(X, Q[idx], a, s, 7)
        out["samples"][str(s)] = {"wall_ms": (t1 - t0) * 1e3, "queries_per_s": m / (t1 - t0),
                                  "kernels_ms": {k: v[1] for k, v in tm.items()},
                                  "mean_rel_err_vs_exact": float(rel.mean()), "max_rel_err_vs_exact": float(rel.max()),
                                  "frac_within_10pct": float(np.mean(rel <= 0.1)),
                                  "max_rel_diff_vs_oracle_estimator": float(np.max(np.abs(Sh[idx] - ref) / ref))}
    return out


def e2lsh_table_run(stag, torch, dev, lib, buf, Xd, Qd, K: int = 6, L: int = 50):
    """E2LSH table (K = 6, L = 50, the paper's example) over the step's data:
    build and near-neighbour listing of all queries, with kernel times."""
    import synth
    n, d = Xd.shape
    m = Qd.shape[0]
    G, b = synth.e2lsh_randomness(K * L, d, 3002)
    Gd, bd = torch.from_numpy(G).to(dev), torch.from_numpy(b).to(dev)
    t = stag.E2LSHTable(Xd, Gd, bd, K, L)  # warm-up
    t.near_neighbours(Qd)
    t.close()
    torch.cuda.synchronize()
    lib.stag_timing_report(buf, len(buf))
    lib.stag_timing_enable(1)
    t0 = time.perf_counter()
    t = stag.E2LSHTable(Xd, Gd, bd, K, L)
    t1 = time.perf_counter()
    off, idx = t.near_neighbours(Qd)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    lib.stag_timing_enable(0)
    lib.stag_timing_report(buf, len(buf))
    t.close()
    tm = parse_timing(buf.value.decode())
    total = int(off[-1].item())
    ms = {k: v[1] for k, v in tm.items()}
    return {"workload": f"E2LSH table K={K}, L={L} over n={n} points, d={d}; near neighbours of m={m} queries",
            "build_wall_ms": (t1 - t0) * 1e3, "query_wall_ms": (t2 - t1) * 1e3,
            "kernels_ms": ms, "neighbours_per_query": total / m,
            "queries_per_s": m / (t2 - t1), "listed_per_s": total / (t2 - t1)}


def serving_run(stag, torch, dev, n_requests: int, seconds_cap: float, eps: float = 1e-3, lsh_share: float = 0.1,
                cmp_requests: int = 600, cmp_eps: float = 3e-3):
    """Requests of log-uniform size (1..65536) against four resident data
    sets, each held in fp32 (centred tiles), bf16 split and fp16 split with a
    CKNS index.  Mixed stream: exact requests with a stated accuracy eps (the
    form chosen per request by the STAG_FORM_AUTO rule) and a share of LSH
    requests; a burst submitted at once measures the saturation throughput,
    then Poisson streams of n_requests requests at 0.5, 0.8 and 0.95 of the
    saturation request rate give latency percentiles (overall and per form)
    and throughput (0.5 is the headline figure).  Equal-accuracy comparison
    at the stated accuracy cmp_eps (the bf16 split form's largest bound on
    these data sets is about 2e-3): the same exact requests in the fp32, bf16
    split and fp16 split forms, each as a burst (saturation) and as a Poisson
    stream at half of the fp32 saturation rate, with the largest bound seen.  Each request's queries are a
    contiguous slice of a resident pool of 65,536 draws from its data set's
    mixture (no host traffic per request)."""
    import numpy as np

    import synth
    specs = [(100_000, 16), (300_000, 64), (1_000_000, 256), (2_000_000, 64)]
    lsh = dict(eps=0.5, k1=1, k2_constant=8, p_offset=1, seed=3005)
    with_index = (0, 1)  # CKNS indexes on the two smaller data sets (the estimator's work grows with n)
    srv = stag.Server(budget_bytes=24 << 30, n_streams=4, max_batch_queries=65536, chunk_queries=4096)
    ids, pools, host = [], [], []
    for k, (n, d) in enumerate(specs):
        mix = synth.mixture(d, 20, 4005 + 10 * k, sigma=(0.5, 2.0))
        Xh = synth.sample(mix, n, 4105 + 10 * k)
        X = torch.from_numpy(Xh).to(dev)
        ids.append(srv.add_dataset(X, 0.64 / d, ["fp32", "bf16_split", "fp16_split"],
                                   lsh=lsh if k in with_index else None))
        pools.append(torch.from_numpy(synth.sample(mix, 65536, 4205 + 10 * k)).to(dev))
        host.append(Xh)
        del X
    torch.cuda.synchronize()
    print("[bench] serving: data sets resident", file=sys.stderr, flush=True)

    def make(count, rate, seed, kinds):
        arr, sizes, dsel = synth.poisson_requests(count, rate_per_s=rate, seed=seed)
        u = np.random.default_rng(seed + 1).random(count)
        reqs = []
        for r in range(count):
            k, mr = int(dsel[r]), int(sizes[r])
            off = (r * 7919) % (65536 - mr + 1)
            if isinstance(kinds, str):
                kind = kinds
            else:
                kind = "lsh" if (k in with_index and u[r] < lsh_share / (len(with_index) / len(specs))) else "auto"
            reqs.append((k, pools[k][off:off + mr], kind))
        return arr, reqs

    def run(arr, reqs, paced):
        t_start = time.perf_counter()
        tickets = []
        for r, (k, Q, kind) in enumerate(reqs):
            if paced:
                now = time.perf_counter() - t_start
                if arr[r] > now:
                    time.sleep(arr[r] - now)
            if time.perf_counter() - t_start > seconds_cap:
                break
            if kind == "lsh":
                t = srv.submit(ids[k], Q, lsh=True)
            else:
                t = srv.submit(ids[k], Q, form=kind, eps=eps, bound=True)
            tickets.append((t, srv.form_of(t) or "lsh", Q.shape[0], specs[k][0]))
        lat, evals, by, bmax = [], 0.0, {}, 0.0
        for t, f, m, n in tickets:
            _, st, l = srv.wait(t)
            B = srv.bound_of(t)
            if st == 0:
                lat.append(l)
                by.setdefault(f, []).append(l)
                if f != "lsh":
                    evals += float(m) * n
                    bmax = max(bmax, float(B.max().item()))
        t_end = time.perf_counter()

        def pct(v, p):
            v = np.sort(np.array(v))
            return float(v[max(0, math.ceil(p / 100 * len(v)) - 1)]) * 1e3 if len(v) else None
        return {"requests": len(tickets), "completed": len(lat), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
                "exact_evals_per_s": evals / (t_end - t_start), "exact_evals": evals, "wall_s": t_end - t_start,
                "max_bound": bmax,
                "per_form": {f: {"requests": len(v), "p50_ms": pct(v, 50), "p99_ms": pct(v, 99)}
                             for f, v in sorted(by.items())}}

    # mixed stream: saturation burst, then three loads
    arr, reqs = make(min(n_requests, 1000), 1.0, 4005, None)
    burst = run(arr, reqs, paced=False)
    req_rate = burst["requests"] / burst["wall_s"]
    print(f"[bench] serving: saturation {req_rate:.1f} requests/s", file=sys.stderr, flush=True)
    loads = []
    for li, rho in enumerate((0.5, 0.8, 0.95)):
        arr, reqs = make(n_requests, rho * req_rate, 4006 + li, None)
        r = run(arr, reqs, paced=True)
        r.update({"rho": rho, "offered_rate_per_s": rho * req_rate})
        loads.append(r)
        print(f"[bench] serving: load {rho} p50 {r['p50_ms']:.2f} ms p99 {r['p99_ms']:.2f} ms", file=sys.stderr,
              flush=True)
    # equal stated accuracy: fp32 vs bf16 split, exact requests only
    cmp = {}
    cmp_forms = ("fp32", "bf16_split", "fp16_split")
    arr_b, reqs_b = make(min(cmp_requests, 400), 1.0, 4010, "x")
    for form in cmp_forms:
        rb = run(arr_b, [(k, Q, form) for k, Q, _ in reqs_b], paced=False)
        cmp[form] = {"saturation_exact_evals_per_s": rb["exact_evals_per_s"],
                     "saturation_request_rate_per_s": rb["requests"] / rb["wall_s"], "max_bound": rb["max_bound"]}
    print("[bench] serving: equal-accuracy bursts done", file=sys.stderr, flush=True)
    rate32 = 0.5 * cmp["fp32"]["saturation_request_rate_per_s"]
    arr_c, reqs_c = make(cmp_requests, rate32, 4011, "x")
    for form in cmp_forms:
        r = run(arr_c, [(k, Q, form) for k, Q, _ in reqs_c], paced=True)
        cmp[form].update({"load": {"offered_rate_per_s": rate32, "requests": r["requests"], "p50_ms": r["p50_ms"],
                                   "p99_ms": r["p99_ms"], "exact_evals_per_s": r["exact_evals_per_s"],
                                   "max_bound": r["max_bound"]}})
    cmp["stated_accuracy"] = cmp_eps
    cmp["all_within_stated_accuracy"] = bool(max(cmp[f]["max_bound"] for f in cmp_forms) <= cmp_eps)
    cmp["bf16_split_over_fp32_saturation"] = (cmp["bf16_split"]["saturation_exact_evals_per_s"] /
                                              cmp["fp32"]["saturation_exact_evals_per_s"])
    # accuracy of served results against the FP64 oracle: 32 queries per data
    # set at the stream's eps (AUTO) and in each compared form
    import oracle
    check = {}
    for form in ("auto",) + cmp_forms:
        worst, wb = 0.0, 0.0
        for k, (n, d) in enumerate(specs):
            Q = pools[k][1000:1032]
            t = srv.submit(ids[k], Q, form=form, eps=eps if form == "auto" else cmp_eps, bound=True)
            S, st, _ = srv.wait(t)
            B = srv.bound_of(t).cpu().numpy()
            ref = oracle.kde_exact(host[k], Q.cpu().numpy(), 0.64 / d)
            err = np.abs(S.cpu().numpy() - ref) / ref
            worst, wb = max(worst, float(err.max())), max(wb, float((err / B).max()))
        check[form] = {"max_rel_err": worst, "max_err_over_bound": wb}
    print("[bench] serving: oracle check done", file=sys.stderr, flush=True)
    stats = srv.stats()
    srv.close()
    head = loads[0]
    return {"p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"], "exact_evals_per_s": head["exact_evals_per_s"],
            "headline_load": 0.5, "stated_accuracy": eps, "lsh_share": lsh_share,
            "saturation": burst, "saturation_request_rate_per_s": req_rate, "loads": loads,
            "equal_accuracy_forms": cmp, "oracle_check_32_queries_per_dataset": check,
            "completed": int(stats["completed"]),
            "batches": int(stats["batches"]), "datasets": [f"n={n} d={d}" for n, d in specs],
            "resident_forms": ["fp32 (centred)", "bf16_split", "fp16_split"], "lsh_index": lsh,
            "chunk_queries": 4096, "batch_sizes": "log-uniform 1..65536", "requests_per_load": n_requests}


HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILES = [os.path.join(HERE, "profiles", "exact_tile_n2m_q200k_d128_hbm_traffic.txt"),
                 os.path.join(HERE, "profiles", "hot_path_step_n100k_d64_hbm_traffic.txt")]
CSRC = os.path.join(HERE, "paper_2407_07096_amd", "csrc")
TRAFFIC_SOURCES = {"kde_tile": ["kde_tiles.h", "kde_tiles_gauss.hip", "kde_tiles_gauss_extra.hip", "kde_exact.h"],
                   "lsh_": ["lsh.hip", "e2lsh.h"], "simgraph_draw": ["simgraph.hip"]}


def committed_traffic(key, workload_tag):
    """HBM bytes per launch of a kernel from a committed counter summary
    (FETCH_SIZE/WRITE_SIZE scaled by the copy calibration), or None when no
    summary of that workload has an entry or the kernel's sources changed
    since it was taken."""
    import hashlib
    srcs = next((v for k, v in TRAFFIC_SOURCES.items() if key.startswith(k)), None)
    if srcs is None:
        return None
    h = hashlib.sha256()
    for f in srcs:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    cur = h.hexdigest()[:16]
    for path in TRAFFIC_FILES:
        if not os.path.exists(path) or workload_tag not in os.path.basename(path):
            continue
        with open(path) as fh:
            for line in fh:
                parts = line.split()
                if len(parts) == 6 and parts[0] == key and not line.startswith("#"):
                    return float(parts[5]) if parts[2] == cur else None
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--form", default="fp16_adaptive", choices=sorted(MFMA_PEAK))
    ap.add_argument("--check-queries", type=int, default=1000)
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline (and the CPU baseline unless --no-cpu-baseline)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only-step", action="store_true",
                    help="profiling aid: only the hot-path step at n = m = 1e5, d = 64 (its JSON object alone)")
    ap.add_argument("--only-edge-sampling", action="store_true",
                    help="profiling aid: only the 784-dimensional edge sampling (n = 70,000; its JSON object alone)")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="after the timed steps, one plain device copy of this many MiB (a reference for "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported.  Over several GPUs the exact "
              "KDE would split X by rows (one fp64 sum all-reduce of the m results), the CKNS estimator its "
              "independent copies, and the edge sampler its nodes with X replicated", file=sys.stderr)
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
    buf = ctypes.create_string_buffer(1 << 16)
    dev = torch.device("cuda:0")

    if args.only_step:
        X, Q, info = synth.config_points(2)
        Xd = torch.from_numpy(X).to(dev)
        Qd = torch.from_numpy(Q).to(dev)
        step, _ = hot_path_step_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, STEP_FORM, 0.01, steps=args.steps)
        if args.calib_copy_mb > 0:
            src_c = torch.ones(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
            dst_c = torch.empty_like(src_c)
            torch.cuda.synchronize()
            torch.mul(src_c, 1.0, out=dst_c)
            torch.cuda.synchronize()
        print(json.dumps({"hot_path_step": step}), flush=True)
        return

    if args.only_edge_sampling:
        c4 = c4_run(stag, torch, dev, lib, buf, C4_LSH)
        print(json.dumps({"edge_sampling_784d": c4}), flush=True)
        return

    # ---- headline: exact KDE, n = 2e6, m = 2e5, d = 128 ----
    X3, Q3, info3 = synth.config_points(3)
    n, d, m = info3["n"], info3["d"], info3["m"]
    a = HEADLINE_A
    Xd = torch.from_numpy(X3).to(dev)
    Qd = torch.from_numpy(Q3).to(dev)
    S = torch.empty(m, dtype=torch.float64, device=dev)
    print(f"[bench] headline data ready: n={n} m={m} d={d}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        stag.kde_exact(Xd, Qd, a, form=args.form, S_out=S)
    with Timers(lib, buf, torch) as tm:
        for _ in range(args.steps):
            stag.kde_exact(Xd, Qd, a, form=args.form, S_out=S)
    ms_per_step = tm.wall_s * 1e3 / args.steps
    evals = float(n) * m
    value = evals / (ms_per_step / 1e3)
    per_step = {k: v[1] / args.steps for k, v in tm.t.items()}
    print(f"[bench] headline {ms_per_step:.2f} ms/step", file=sys.stderr, flush=True)
    if args.calib_copy_mb > 0:
        src_c = torch.ones(args.calib_copy_mb << 18, dtype=torch.float32, device=dev)
        dst_c = torch.empty_like(src_c)
        torch.cuda.synchronize()
        torch.mul(src_c, 1.0, out=dst_c)  # one streaming kernel: reads and writes calib bytes
        torch.cuda.synchronize()
        del src_c, dst_c
    tk = TILE_KERNEL[args.form]
    c, tot = tm.t[tk]
    tile_avg = tot / c
    useful = 2.0 * d * evals
    roof = {"bound": "mfma", "achieved": useful / (tile_avg / 1e3) / 1e12, "peak": MFMA_PEAK[args.form] / 1e12,
            "unit": "TFLOP/s", "frac": useful / (tile_avg / 1e3) / MFMA_PEAK[args.form],
            "traffic": committed_traffic(tk, "n2m_q200k_d128"), "kernel": tk, "avg_launch_ms": tile_avg,
            "launches_per_step": c / args.steps,
            "frac_hardware": useful * PRODUCTS[args.form] / (tile_avg / 1e3) / MFMA_PEAK[args.form],
            "algorithmic": f"2*d = {2 * d} flops per (query, point) pair x n*m = {useful:.4e} per launch (the "
                           f"method's work); the {args.form} form issues {PRODUCTS[args.form]} matrix-core "
                           f"products per pair (frac_hardware)"}
    if args.form == "fp16_adaptive" and "kde_tile_fp16x3" in tm.t:
        c2, tot2 = tm.t["kde_tile_fp16x3"]
        roof["second_pass"] = {"kernel": "kde_tile_fp16x3", "avg_launch_ms": tot2 / c2,
                               "what": "the fp16 split tiles over the selected (chunk, 256-query tile) pairs; "
                                       "the other workgroups of its grid return at once"}
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
        "dtype": DTYPE[args.form],
        "data": "synthetic",
        "config": {"workload": f"exact Gaussian KDE, n={n} data, m={m} queries, d={d}, 50-component isotropic "
                               f"mixture (means U[-5,5]^d, sigma U[0.5,2]), a={a}, form {args.form}; one step = "
                               f"one call over all queries, inputs resident in HBM",
                   "n": n, "m": m, "d": d, "a": a, "form": args.form},
        "exact_kde_ms_per_step": ms_per_step,
        "kernels_ms_per_step": per_step,
        "roofline": roof,
    }
    if args.check_queries > 0:
        rng = np.random.default_rng(2003)
        idx = np.sort(rng.choice(m, size=args.check_queries, replace=False))
        t0 = time.perf_counter()
        ref = oracle_reference(X3, Q3, idx, a)
        t_ref = time.perf_counter() - t0
        err = np.abs(S.cpu().numpy()[idx] - ref) / ref
        result["max_rel_err_sampled"] = float(err.max())
        result["median_rel_err_sampled"] = float(np.median(err))
        result["checked_queries"] = int(args.check_queries)
        result["oracle_check_s"] = t_ref
        print(f"[bench] checked {args.check_queries} queries: max rel err {err.max():.3e}", file=sys.stderr,
              flush=True)
        if not args.no_extras:
            others = [f for f in ("fp16_split", "fp16_centred", "bf16_split", "bf16_split3", "fp32") if f != args.form]
            result["forms"] = forms_run(stag, torch, lib, buf, Xd, Qd, a, idx, ref, others, n, m, d)
            print("[bench] other forms done", file=sys.stderr, flush=True)
            result["lsh_headline_workload"] = lsh_headline_run(stag, torch, lib, buf, Xd, Qd, a, idx, ref, ms_per_step)
            print("[bench] CKNS on the headline workload done", file=sys.stderr, flush=True)
            result["headline_a_0.001"] = second_bandwidth_run(stag, torch, lib, buf, X3, Q3, Xd, Qd, idx, args.form,
                                                              0.001)
            print("[bench] headline workload at a = 0.001 done", file=sys.stderr, flush=True)
    del Xd, Qd, S
    torch.cuda.empty_cache()

    if not args.no_extras:
        X, Q, info = synth.config_points(2)
        Xd = torch.from_numpy(X).to(dev)
        Qd = torch.from_numpy(Q).to(dev)
        a2 = 0.01
        step, graph = hot_path_step_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, STEP_FORM, a2, steps=5)
        result["hot_path_step"] = step
        for k, v in result["hot_path_step"]["rooflines"].items():
            v["traffic"] = committed_traffic(k, "n100k_d64")
        print("[bench] hot-path step done", file=sys.stderr, flush=True)
        result["lsh_default_parameters"] = lsh_defaults_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, a2)
        print("[bench] CKNS defaults done", file=sys.stderr, flush=True)
        result["e2lsh_table"] = e2lsh_table_run(stag, torch, dev, lib, buf, Xd, Qd)
        result["kernels"] = kernels_run(stag, torch, dev, lib, buf, X, Q, Xd, Qd, STEP_FORM)
        result["random_sampling"] = rs_run(stag, torch, lib, buf, X, Q, Xd, Qd, a2, STEP_FORM)
        result["spectral"] = spectral_run(stag, torch, lib, buf, graph, info["n"], info["k"], info["labels"])
        result["kde_tree_sampler"] = tree_run(stag, torch, lib, buf, X, Xd, a2, graph, info["labels"], info["k"])
        del graph, Xd, Qd
        torch.cuda.empty_cache()
        print("[bench] step extras done", file=sys.stderr, flush=True)
        result["edge_sampling_784d"] = c4_run(stag, torch, dev, lib, buf, C4_LSH)
        print("[bench] 784-d edge sampling done", file=sys.stderr, flush=True)
        if not args.no_serve:
            result["serving"] = serving_run(stag, torch, dev, args.serve_requests, seconds_cap=90.0)
            print("[bench] serving done", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(X3, Q3, a, args.cpu_budget)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

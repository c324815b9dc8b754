#!/usr/bin/env python3
"""Benchmark: IPM time-to-certificate at duality gap 1e-8 on one MI355X.

One step = the whole hot path over one batch of synthetic input: Polya
set-up of every system (vertices already resident in HBM), the batched
predictor-corrector interior-point solve to relative gap 1e-8 (Schur
complement assembly, its FP64 Cholesky and solves, the step-length ladder,
updates; phase-I for undecided systems) and the FP64 block-Cholesky
certificate check.  The default workload is 64 seeded uncertain systems with
n=10 states, l=4 vertices, dp=2, d=2 (K=550 unknowns, 35 + 56 blocks each).

Prints one JSON line; see the design notes for the roofline definitions.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload n10|n100]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IPM time-to-certificate @gap 1e-8: FP64 vs mixed/warm-start; Schur TFLOP/s"
PEAK_FP64 = 78.6          # TFLOP/s, FP64 vector and FP64 matrix (MI355X)
PEAK_HBM = 8000.0         # GB/s


def _mons(l, d):
    out = []

    def rec(prefix, rem):
        if len(prefix) == l - 1:
            out.append(tuple(prefix + [rem]))
            return
        for v in range(rem, -1, -1):
            rec(prefix + [v], rem - v)
    rec([], d)
    return out


def schur_flops(n, l, dp, d):
    """Algorithmic flops of one Schur complement assembly (structured
    expansion; one triangle): (Nt^2 / 2) (8 sum_j n_j^2 + 32 sum_m z_m^2),
    n_j / z_m = number of P_h coefficients present in block j / m."""
    Wp, WL, WM = _mons(l, dp), _mons(l, dp + d), _mons(l, dp + 1 + d)
    ge = lambda g, h: all(a >= b for a, b in zip(g, h))
    nj = [sum(ge(g, h) for h in Wp) for g in WL]
    zm = [sum(ge(g, h) for h in Wp) for g in WM]
    Nt = n * (n + 1) // 2
    return Nt * Nt / 2.0 * (8 * sum(x * x for x in nj) + 32 * sum(x * x for x in zm))


def workload(name):
    from paper_1411_3769_amd import workloads as W
    if name == "n10":
        return [W.c1_system(s) for s in range(64)], "n10 l4 dp2 d2, 64 seeds (K=550)"
    if name == "n100":
        return [W.c2_system(0)], "n100 l4 dp1 d3, seed 0 (K=20200)"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(systems, budget_s=15.0):
    """The oracle, untuned, on the host: full solves of the first seeds of the
    workload until about budget_s of CPU time, extrapolated to the batch."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:       # pragma: no cover
        threadpool_limits = None
    from oracle import ipm, sdp as S
    ctx = threadpool_limits(1) if threadpool_limits else None
    t0 = time.perf_counter()
    done = 0
    try:
        for sy in systems:
            ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d))
            done += 1
            if time.perf_counter() - t0 > budget_s:
                break
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    el = time.perf_counter() - t0
    return dict(value=el / done * len(systems), unit="s", cores=1, kind="oracle",
                sample=f"{done} of {len(systems)} systems solved by the FP64 oracle "
                       f"({el:.1f} s, one thread), scaled by {len(systems)}/{done}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n10")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: this build has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1411_3769_amd import polyaipm as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.load()
    systems, desc = workload(args.workload)
    # inputs resident in HBM before the timed region
    A_dev = [torch.tensor(sy.A, device="cuda:0", dtype=torch.float64) for sy in systems]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream

    def step(prof=None):
        hs = [P.polya_setup(A, sy.n, sy.l, sy.dp, sy.d) for A, sy in zip(A_dev, systems)]
        rs = P.ipm_solve_batched(hs, stream=stream, prof=prof)
        for h in hs:
            h.close()
        return rs

    for _ in range(args.warmup):
        step()
    prof = P.new_prof()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        results.append(step(prof))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms = el / args.steps * 1e3
    rs = results[-1]
    verdicts = {}
    for r in rs:
        verdicts[r.verdict_name] = verdicts.get(r.verdict_name, 0) + 1

    # roofline of the dominant launch class (device time from HIP events)
    per = {P.PROF_CLASSES[i]: (prof[i, 0], prof[i, 1]) for i in range(len(P.PROF_CLASSES))}
    dom = max(per, key=lambda k: per[k][0])
    iters_sys = [r.iterations for r in rs]
    asm_flops = sum(it * schur_flops(sy.n, sy.l, sy.dp, sy.d) for it, sy in zip(iters_sys, systems))
    from math import comb
    Ks = [comb(sy.l + sy.dp - 1, sy.l - 1) * sy.n * (sy.n + 1) // 2 for sy in systems]
    chol_flops = sum(it * k ** 3 / 3.0 for it, k in zip(iters_sys, Ks))
    asm_ms = per["assemble"][0] / args.steps
    chol_ms = (per["chol_panel"][0] + per["chol_update"][0]) / args.steps
    asm_tf = asm_flops / (asm_ms * 1e-3) / 1e12 if asm_ms > 0 else None
    chol_tf = chol_flops / (chol_ms * 1e-3) / 1e12 if chol_ms > 0 else None
    launches = per[dom][1] / args.steps
    avg_ms = per[dom][0] / max(per[dom][1], 1)
    if dom == "assemble":
        per_launch = asm_flops / max(launches, 1)
        roof = dict(bound="alu", achieved=per_launch / (avg_ms * 1e-3) / 1e12, peak=PEAK_FP64,
                    unit="TFLOP/s", kernel="k_assemble (Schur complement assembly, FP64 FMA)")
    elif dom in ("chol_update", "chol_panel"):
        roof = dict(bound="alu", achieved=chol_tf, peak=PEAK_FP64, unit="TFLOP/s",
                    kernel="k_chol_panel + k_chol_update (Schur Cholesky, FP64 FMA)")
    else:
        roof = dict(bound="alu", achieved=None, peak=PEAK_FP64, unit="TFLOP/s", kernel=dom)
    roof["frac"] = (roof["achieved"] / roof["peak"]) if roof.get("achieved") else None
    roof["traffic"] = None
    roof["avg_launch_ms"] = avg_ms
    roof["launches_per_step"] = launches

    line = {
        "metric": METRIC,
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded dissipative systems, see workloads.py)",
        "config": {"workload": desc, "systems": len(systems), "gap_tol": 1e-8,
                   "verdicts": verdicts, "iterations_mean": float(np.mean(iters_sys)),
                   "schur_assembly_tflops": asm_tf, "schur_cholesky_tflops": chol_tf,
                   "device_ms_per_step": {k: round(v[0] / args.steps, 3) for k, v in per.items()}},
        "roofline": roof,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(systems)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

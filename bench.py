#!/usr/bin/env python3
"""Benchmark: IPM time-to-certificate at duality gap 1e-8 on one MI355X.

One step = the whole hot path over one batch of synthetic input: Polya
set-up of every system (vertices already resident in HBM), the batched
predictor-corrector interior-point solve to relative gap 1e-8 (Schur
complement assembly, its FP64 Cholesky and solves, the step-length ladder,
updates; phase-I for undecided systems) and the FP64 block-Cholesky
certificate check.

The default workload is the single large system n=100, l=4, dp=1, d=3
(K = 20200 unknowns, a 20200 x 20200 Schur complement): `value` is its FP64
time-to-certificate; the same line carries the precision forms (Schur
assembly in FP32 and in BF16 on MFMA, FP64 Cholesky, refinement against the
FP64 matrix-free product), each with its error against the stored FP64
oracle end point, the roofline of the dominant kernel group (the Schur
Cholesky) and the oracle's own time on the host.  Other workloads: n10 (64
systems n=10, l=4, dp=d=2, K=550), mixed512 (the uneven batch of 512),
learned (warm start on the n=32 family).

Prints one JSON line; see the design notes for the roofline definitions.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload n100|n10|mixed512|learned]
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IPM time-to-certificate @gap 1e-8: FP64 vs mixed/warm-start; Schur TFLOP/s"
PEAK_FP64 = 78.6          # TFLOP/s, FP64 vector and FP64 matrix (MI355X)
PEAK_HBM = 8000.0         # GB/s

# HBM bytes per launch of the dominant kernel group, from the two rocprofv3
# --pmc runs summarised in profiles/hbm_counters_n10_batch64.md and
# profiles/hbm_counters_n100_fp64.md (FETCH_SIZE
# and WRITE_SIZE in KiB per dispatch over the group's dispatches, scaled by
# what they read for a plain 256 MiB device copy: x2.000 and x1.000).  Valid
# for the kernel versions those runs measured; drop an entry once they change.
PMC_TRAFFIC = {
    # n = 10: one super-panel (8 or 16 panels give the same launches at 9 tiles)
    ("n10", "cholesky"): dict(fetch_kib=21931.3, fetch_scale=2.000, write_kib=17995.3, write_scale=1.000,
                              widths={8, 16}, dispatches_per_step=1411 / 3),
    ("n100", "cholesky"): dict(fetch_kib=49848.5, fetch_scale=2.000, write_kib=34763.7, write_scale=1.000,
                               widths={16}, dispatches_per_step=35964 / 2),
}


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


def schur_flops(n, l, dp, d, form="continuous"):
    """Algorithmic flops of one Schur complement assembly (structured
    expansion; one triangle): (Nt^2 / 2) (8 sum_j n_j^2 + 32 sum_m z_m^2),
    n_j / z_m = number of P_h coefficients present in block j / m; the
    discrete form's basis matrices sit on two diagonal copies, so each term
    becomes four (copy pairs) of the same size."""
    Wp, WL, WM = _mons(l, dp), _mons(l, dp + d), _mons(l, dp + 1 + d)
    ge = lambda g, h: all(a >= b for a, b in zip(g, h))
    nj = [sum(ge(g, h) for h in Wp) for g in WL]
    zm = [sum(ge(g, h) for h in Wp) for g in WM]
    Nt = n * (n + 1) // 2
    return (4.0 if form == "discrete" else 1.0) * Nt * Nt / 2.0 * (
        8 * sum(x * x for x in nj) + 32 * sum(x * x for x in zm))


def workload(name):
    from paper_1411_3769_amd import workloads as W
    if name == "n10":
        return [W.c1_system(s) for s in range(64)], "n10 l4 dp2 d2, 64 seeds (K=550)"
    if name == "n100":
        return [W.c2_system(0)], "n100 l4 dp1 d3, seed 0 (K=20200)"
    if name == "mixed512":
        return W.mixed_systems(512), "mixed batch of 512: n 6..48, l 2..5, dp 1..2, d 1..4 (K 42..17640)"
    if name == "discrete":
        return ([W.discrete_system(s) for s in range(64)],
                "discrete time x+ = A(alpha) x: n8 l4 dp1 d1, 64 contractive seeds (K=144, blocks of order 16)")
    raise SystemExit(f"unknown workload {name}")


def host_threads():
    """Host threads the oracle may use: this process's CPU affinity set, capped
    by OMP_NUM_THREADS when it is set (a host shared with other jobs sets it to
    its share)."""
    n = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return n


def _limits(threads):
    try:
        from threadpoolctl import threadpool_limits
        return threadpool_limits(threads)
    except Exception:       # pragma: no cover
        import contextlib
        return contextlib.nullcontext()


def _oracle_sdp(A, n, l, dp, d, form):
    from oracle import discrete as Dd, sdp as S
    return (Dd.make_discrete_sdp if form == "discrete" else S.make_sdp)(A, n, l, dp, d)


def _oracle_solve(args):
    """One full FP64 oracle solve on one host thread (a pool worker)."""
    A, n, l, dp, d, form = args
    from oracle import ipm
    with _limits(1):
        ipm.ipm_solve(_oracle_sdp(A, n, l, dp, d, form))
    return 1


def cpu_baseline_solves(systems, budget_s, threads):
    """The oracle, untuned, on the host: full solves of the workload's systems
    until about budget_s of wall time, extrapolated to the batch.  With more
    than one thread, one system per worker process (each on one BLAS thread)
    over `threads` processes, started fresh (spawn: nothing of this process's
    GPU state is inherited)."""
    from oracle import ipm
    t0 = time.perf_counter()
    done = 0
    if threads <= 1:
        with _limits(1):
            for sy in systems:
                ipm.ipm_solve(_oracle_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d, sy.form))
                done += 1
                if time.perf_counter() - t0 > budget_s:
                    break
        el = time.perf_counter() - t0
        desc = "1 thread"
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=threads, mp_context=mp.get_context("spawn")) as ex:
            # workers started and warm before the clock runs
            list(ex.map(int, range(threads)))
            t0 = time.perf_counter()
            futs = [ex.submit(_oracle_solve, (sy.A, sy.n, sy.l, sy.dp, sy.d, sy.form)) for sy in systems]
            for f in cf.as_completed(futs):
                done += f.result()
                if time.perf_counter() - t0 > budget_s:
                    break
            el = time.perf_counter() - t0
            for f in futs:
                f.cancel()
        desc = f"{threads} worker processes of one thread each"
    return dict(value=el / done * len(systems), unit="s", cores=threads, kind="oracle",
                sample=f"{done} of {len(systems)} systems solved by the FP64 oracle "
                       f"({el:.1f} s, {desc}), scaled by {len(systems)}/{done}")


def cpu_baseline_iteration(sy, iterations, threads):
    """The oracle on the large system: its set-up plus one interior-point
    iteration (expanded-mode Schur complement, LAPACK Cholesky, both solves,
    directions, ladders, residuals) timed on `threads` host threads, the
    iteration scaled by the GPU solve's iteration count."""
    from oracle import ipm, sdp as S
    with _limits(threads):
        t0 = time.perf_counter()
        sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
        t1 = time.perf_counter()
        ipm.ipm_run(ipm.PaperOps(sdp), ipm.Options(), max_iter=1)
        t2 = time.perf_counter()
    return dict(value=(t1 - t0) + (t2 - t1) * iterations, unit="s", cores=threads, kind="oracle",
                sample=f"the FP64 oracle's set-up ({t1 - t0:.1f} s) and one IPM iteration "
                       f"({t2 - t1:.1f} s) of the K=20200 system on {threads} host threads, the "
                       f"iteration scaled by the GPU run's {iterations} iterations")


def oracle_end_point(sy):
    """Stored FP64 oracle end point of a large system (written by
    tests/golden/make_oracle_results.py --large), or None."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_results_large.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for rec in json.load(fh):
            if rec["tag"] == sy.tag and rec["seed"] == sy.seed:
                return rec
    return None


def error_vs_oracle(r, rec):
    if rec is None:
        return None
    rel = lambda a, b: abs(a - b) / abs(b) if b else None
    return {"verdict_equal": r.verdict_name == rec["verdict"],
            "psi_rel": rel(r.psi, rec["psi"]), "phi_rel": rel(r.phi, rec["phi"]),
            "margin_rel": rel(r.margin, rec["margin"]),
            "iterations": r.iterations, "oracle_iterations": rec["iterations"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n100", help="n100 | n10 | mixed512 | discrete | learned | example2")
    ap.add_argument("--precision", default=None, help="fp64 | fp32 | bf16 (Schur assembly)")
    ap.add_argument("--form-steps", type=int, default=3,
                    help="n100: timed steps of each precision form (at most --steps)")
    ap.add_argument("--no-forms", action="store_true", help="n100: skip the precision forms")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch every kernel eagerly")
    ap.add_argument("--chol-panels", type=int, default=0,
                    help="Schur Cholesky: -1 left-looking, 1..32 super-panel width, 0 autotuned")
    ap.add_argument("--chol-subpanels", type=int, default=0,
                    help="with --chol-panels w: sub-panels of this width (a divisor of w), 0 none")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy 3 times (reference for HBM counters)")
    ap.add_argument("--train", type=int, default=20000, help="learned: training solves")
    ap.add_argument("--test", type=int, default=2000, help="learned: held-out solves")
    ap.add_argument("--epochs", type=int, default=60, help="learned: training epochs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1411_3769_amd import polyaipm as P

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    P.load()
    log = lambda m: print(m, file=sys.stderr, flush=True)
    if args.calibrate_copy:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "example2":
        return bench_example2(args)
    big = args.workload == "n100"
    prec = args.precision or ("fp32" if args.workload == "mixed512" else "fp64")
    systems, desc = workload(args.workload)
    # inputs resident in HBM before the timed region
    A_dev = [torch.tensor(sy.A, device="cuda:0", dtype=torch.float64) for sy in systems]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream

    tsplit = [0.0, 0.0]

    def step(precision, prof=None):
        t0 = time.perf_counter()
        hs = P.polya_setup_batched([(A, sy.n, sy.l, sy.dp, sy.d) for A, sy in zip(A_dev, systems)],
                                   form=systems[0].form)
        t1 = time.perf_counter()
        rs = P.ipm_solve_batched(hs, stream=stream, prof=prof, precision=precision,
                                 use_graph=0 if args.no_graph else 1, chol_panels=args.chol_panels,
                                 chol_subpanels=args.chol_subpanels)
        t2 = time.perf_counter()
        for h in hs:
            h.close()
        tsplit[0] += t1 - t0
        tsplit[1] += t2 - t1
        return rs

    def timed(precision, steps, warmup):
        for _ in range(warmup):
            step(precision)
        tsplit[0] = tsplit[1] = 0.0
        quiet_gc()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results = []
        for _ in range(steps):
            results.append(step(precision))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        return el / steps, results[-1], (tsplit[0] / steps, tsplit[1] / steps)

    log(f"{desc}: {prec}, {args.warmup} warm-up + {args.steps} timed steps")
    sec, rs, split = timed(prec, args.steps, args.warmup)
    ms = sec * 1e3
    log(f"  {ms:.1f} ms per step")

    # the precision forms of the large system, fewer steps each
    forms = {}
    if big and not args.no_forms:
        rec = oracle_end_point(systems[0])
        forms["fp64"] = {"s": sec, "steps": args.steps, "iterations": rs[0].iterations,
                         "verdict": rs[0].verdict_name, "error_vs_oracle": error_vs_oracle(rs[0], rec)}
        for fp in ("fp32", "bf16"):
            k = max(1, min(args.form_steps, args.steps))
            log(f"  form {fp}: 1 warm-up + {k} timed steps")
            fs, frs, _ = timed(fp, k, 1)
            r = frs[0]
            forms[fp] = {"s": fs, "steps": k, "iterations": r.iterations,
                         "lowprec_iterations": r.iters_lowprec, "refinement_steps": r.ir_steps,
                         "ir_eta_max": r.ir_eta_max if r.ir_eta_max == r.ir_eta_max else None,
                         "verdict": r.verdict_name, "vs_fp64": fs / sec,
                         "error_vs_oracle": error_vs_oracle(r, rec)}
            log(f"    {fs * 1e3:.1f} ms, {r.iters_lowprec} of {r.iterations} iterations in {fp}")

    # Per-class device times: HIP events on the solver stream around each
    # launch class, in a profiled pass of the same steps run after the timed
    # region (events recorded inside hipGraphs carry no timestamps, so this
    # pass launches eagerly; kernel durations are unchanged).
    psteps = 1 if big else args.steps
    prof = P.new_prof()
    torch.cuda.synchronize()
    tp = time.perf_counter()
    for _ in range(psteps):
        step(prec, prof)
    torch.cuda.synchronize()
    prof_ms = (time.perf_counter() - tp) / psteps * 1e3
    verdicts = {}
    for r in rs:
        verdicts[r.verdict_name] = verdicts.get(r.verdict_name, 0) + 1

    # roofline of the dominant launch class (device time from HIP events); the
    # Cholesky's two classes (diagonal + panel steps, updates) count as one
    per = {P.PROF_CLASSES[i]: (prof[i, 0], prof[i, 1]) for i in range(len(P.PROF_CLASSES))}
    grp = {k: v for k, v in per.items() if k not in ("chol_panel", "chol_update")}
    grp["cholesky"] = (per["chol_panel"][0] + per["chol_update"][0],
                       per["chol_panel"][1] + per["chol_update"][1])
    dom = max(grp, key=lambda k: grp[k][0])
    iters_sys = [r.iterations for r in rs]
    its_all = [r.iterations + r.phase1_iterations for r in rs]
    asm_flops = sum(it * schur_flops(sy.n, sy.l, sy.dp, sy.d, sy.form) for it, sy in zip(its_all, systems))
    from math import comb
    Ks = [comb(sy.l + sy.dp - 1, sy.l - 1) * sy.n * (sy.n + 1) // 2 for sy in systems]
    chol_flops = sum(it * k ** 3 / 3.0 for it, k in zip(its_all, Ks))
    # both triangular sweeps read the factor's lower triangle once: 8 K^2 / 2
    # bytes each, two solves per iteration
    solve_bytes = sum(it * 2 * 2 * 8.0 * k * k / 2 for it, k in zip(its_all, Ks))
    asm_ms = per["assemble"][0] / psteps
    chol_ms = (per["chol_panel"][0] + per["chol_update"][0]) / psteps
    trsv_ms = per["trsv"][0] / psteps
    asm_tf = asm_flops / (asm_ms * 1e-3) / 1e12 if asm_ms > 0 else None
    chol_tf = chol_flops / (chol_ms * 1e-3) / 1e12 if chol_ms > 0 else None
    trsv_gbs = solve_bytes / (trsv_ms * 1e-3) / 1e9 if trsv_ms > 0 else None
    launches = grp[dom][1] / psteps
    avg_ms = grp[dom][0] / max(grp[dom][1], 1)
    if dom == "assemble":
        per_launch = asm_flops / max(launches, 1)
        roof = dict(bound="mfma", achieved=per_launch / (avg_ms * 1e-3) / 1e12, peak=PEAK_FP64,
                    unit="TFLOP/s",
                    kernel="k_assemble_pair / k_assemble_grp (Schur complement assembly, FP64 MFMA)")
    elif dom == "cholesky":
        roof = dict(bound="mfma", achieved=chol_tf, peak=PEAK_FP64, unit="TFLOP/s",
                    kernel="k_chol_diag + k_chol_trsm + k_chol_update(_wide) + k_chol_left + k_chol_fused + k_chol_look (Schur Cholesky, FP64 MFMA)")
    else:
        roof = dict(bound="mfma", achieved=None, peak=PEAK_FP64, unit="TFLOP/s", kernel=dom)
    roof["frac"] = (roof["achieved"] / roof["peak"]) if roof.get("achieved") else None
    # the device's attainable FP64 matrix-core rate (register-only MFMA chains)
    att = P.fp64_mfma_rate(stream)
    roof["attainable"] = att
    roof["frac_attainable"] = (roof["achieved"] / att) if roof.get("achieved") and att > 0 else None
    tr = PMC_TRAFFIC.get((args.workload, dom)) if prec == "fp64" else None
    if tr and not ({r.chol_panels for r in rs} <= tr["widths"]
                   and all(r.chol_subpanels == r.chol_panels for r in rs)):
        tr = None   # the counters were taken for another factorisation
    roof["traffic"] = (1024.0 * (tr["fetch_kib"] * tr["fetch_scale"] + tr["write_kib"] * tr["write_scale"])
                       if tr else None)
    if tr:
        roof["traffic_unit"] = "bytes per launch (HBM read + write, rocprofv3 counters)"
        # the counters' dispatches per step over the group's device time per step
        roof["traffic_GBps"] = roof["traffic"] * tr["dispatches_per_step"] / (chol_ms * 1e-3) / 1e9
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
        "dtype": "f64" if prec == "fp64" else f"f64 (Schur assembly {prec}, refined)",
        "data": "synthetic (seeded dissipative systems, see workloads.py)",
        "config": {"workload": desc, "systems": len(systems), "gap_tol": 1e-8,
                   "precision": prec,
                   "setup_ms_per_step": split[0] * 1e3, "solve_ms_per_step": split[1] * 1e3,
                   "hip_graph_launches_per_step": rs[0].graph_replays,
                   "phase_seconds_last_step": rs[0].phase_times,
                   "chol_panels": sorted({r.chol_panels for r in rs}),
                   "chol_subpanels": sorted({r.chol_subpanels for r in rs}),
                   "profiled_pass_ms_per_step": prof_ms,
                   "verdicts": verdicts, "iterations_mean": float(np.mean(iters_sys)),
                   "lowprec_iterations_mean": float(np.mean([r.iters_lowprec for r in rs])),
                   "schur_assembly_tflops": asm_tf, "schur_cholesky_tflops": chol_tf,
                   "triangular_solves_GBps": trsv_gbs,
                   "device_ms_per_step": {k: round(v[0] / psteps, 3) for k, v in per.items()}},
        "roofline": roof,
    }
    if forms:
        line["config"]["forms"] = forms
    if not args.no_cpu:
        th = host_threads()
        if big:
            log(f"  oracle: one iteration of the large system on {th} host threads")
            cb = cpu_baseline_iteration(systems[0], its_all[0], th)
            from paper_1411_3769_amd import workloads as W
            log("  oracle: n10 seeds on one thread")
            cb["n10_one_thread"] = cpu_baseline_solves([W.c1_system(s) for s in range(64)], 10.0, 1)
        else:
            cb = cpu_baseline_solves(systems, 15.0, th)
            cb["one_thread"] = cpu_baseline_solves(systems, 10.0, 1)
        line["cpu_baseline"] = cb
    print(json.dumps(line))


def quiet_gc():
    """Collect, then move every object that exists now (imported modules,
    inputs) out of the collector's generations: a cyclic collection that
    falls inside the timed region then scans only what the steps allocate
    instead of torch's whole object graph, a pause of tens of milliseconds."""
    gc.collect()
    gc.freeze()


def bench_example2(args):
    """Section V, Example 2: the certified bound on L (the smallest L with
    stability on S_L = {sum x = 2L + 1, L <= x_i <= 1}) by bisection over
    the translated simplices, Polya degrees dp = 2, d = 4, bracket [-0.5, 0.5]
    to 1e-3.  One step = one whole bisection (set-up and solve of every trial
    on the device, 8 trials per round in one batch); the oracle runs the same
    bisection with one trial per round."""
    import numpy as np
    import torch
    from paper_1411_3769_amd import polyaipm as P
    vals = []
    with open(os.path.join(ROOT, "tests", "golden", "example2_matrices.txt")) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                vals.append([float(v) for v in line.split()])
    mats = np.array(vals).reshape(6, 3, 3)
    # A(x) = A1 x1^3 + A2 x1^2 x2 + A3 x1 x2 x3 + A4 x1 x3^2 + A5 x2^3 + A6 x3^3 on
    # x = G(L) alpha, G(L) = I + L (11^T - I), which maps the simplex onto S_L
    exps = [(3, 0, 0), (2, 1, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 0, 3)]
    G0, G1 = np.eye(3), np.ones((3, 3)) - np.eye(3)
    dp, d, tol, width = 2, 4, 1e-3, 8
    run = lambda: P.bisect_simplex(exps, mats, G0, G1, 3, dp, d, 0.5, -0.5, tol, width=width)
    for _ in range(args.warmup):
        run()
    quiet_gc()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = run()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    line = {
        "metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "the paper's printed Example 2 matrices",
        "config": {"workload": f"Example 2 bisection, dp={dp} d={d}, tol {tol}, {width} trials per round",
                   "L_certified": r.t_cert, "L_bracket_other": r.t_other, "trials": len(r.trials),
                   "paper_L_opt": -0.111},
        "roofline": {"bound": "alu", "achieved": None, "peak": PEAK_FP64, "unit": "TFLOP/s", "frac": None,
                     "traffic": None},
    }
    if not args.no_cpu:
        from oracle import stability as St
        th = host_threads()
        with _limits(th):
            t0 = time.perf_counter()
            o = St.bisect_simplex(exps, mats, G0, G1, 3, dp, d, 0.5, -0.5, tol)
            el = time.perf_counter() - t0
        line["cpu_baseline"] = dict(value=el, unit="s", cores=th, kind="oracle",
                                    sample=f"the oracle's whole bisection ({len(o.trials)} trials, one per "
                                           f"round; certified L {o.t_cert:.6f})")
    print(json.dumps(line))


def bench_learned(args):
    """Learned warm start on the n=32, l=4, dp=1, d=2 family: cold solves
    of the training seeds give the labels, the network is trained on the
    GPU, and the timed steps solve the held-out seeds warm (inference and
    cold fallbacks included).  The held-out cold solves are timed too."""
    import numpy as np
    import torch
    from paper_1411_3769_amd import learned as Lm
    from paper_1411_3769_amd import workloads as W
    log = lambda m: print(m, file=sys.stderr, flush=True)
    tr = [W.warm_system(s) for s in range(args.train)]
    te = [W.warm_system(10**6 + s) for s in range(args.test)]
    t0 = time.perf_counter()
    dtr = Lm.solve_cold(tr, log=log)
    t_label = time.perf_counter() - t0
    t0 = time.perf_counter()
    model = Lm.train(dtr, K=2112, epochs=args.epochs, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    cold_s, warm_s, ev = [], [], None
    quiet_gc()
    for k in range(args.warmup + args.steps):
        dte = Lm.solve_cold(te, log=log)
        ev = Lm.evaluate(model, te, dte, log=log)
        if k >= args.warmup:
            cold_s.append(dte.cold_seconds)
            warm_s.append(ev["warm_seconds"])
    per = lambda v: float(np.mean(v)) / args.test * 256
    line = {
        "metric": METRIC,
        "value": per(warm_s),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * float(np.mean(warm_s)),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (network bf16 with fp32 accumulation)",
        "data": "synthetic (seeded dissipative systems, see workloads.py)",
        "config": {"workload": f"learned warm start, n32 l4 dp1 d2 (K=2112): {args.train} training "
                               f"solves, {args.test} held-out; value = seconds per 256 held-out "
                               f"systems, warm (inference + solve + fallbacks)",
                   "cold_s_per_256": per(cold_s),
                   "warm_iterations_mean": ev["warm_iters_mean"],
                   "cold_iterations_mean": ev["cold_iters_mean"],
                   "fallback_rate": ev["fallback_rate"], "verdicts_agree": ev["verdicts_agree"],
                   "label_seconds": t_label, "train_seconds": t_train, "epochs": args.epochs,
                   "final_train_loss": model.history[-1]},
        "roofline": {"bound": "alu", "achieved": None, "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": None, "traffic": None},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()

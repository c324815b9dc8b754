"""GPU parity at the full sizes (marker: gpu), against the oracle's stored end
points of the large cases (tests/golden/oracle_results_large.json, written by
tests/golden/make_oracle_results.py --large from oracle/ alone):

* the n = 100, l = 4, dp = 1, d = 3 system (K = 20200) in FP64 and in the
  precision forms (Schur assembly in FP32 / BF16, FP64 Cholesky, refinement):
  same verdict, objectives and margin within 1e-6; the measured errors are
  printed for each form;
* held-out members of the n = 32 warm-start family (K = 2112);
* the largest members of the 512-system mixed batch;
* the whole mixed batch in one solve: oracle end points for every member the
  oracle has (small and large), and for every member the properties that
  hold at any size (a^T y = psi; on a spread sample also the certificate's
  blocks through the oracle's operators).
"""
import json
import os
from math import comb

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _large():
    path = os.path.join(GOLDEN, "oracle_results_large.json")
    if not os.path.exists(path):
        return []
    with open(path) as fh:
        return json.load(fh)


def _small_mixed():
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        return {r["index"]: r for r in json.load(fh) if r["tag"].startswith("mixed")}


def _rel(a, b):
    return abs(a - b) / abs(b)


def _check(rec, r, its=1):
    assert r.verdict_name == rec["verdict"], (rec["tag"], r.verdict_name, r.reason_name)
    errs = {}
    if rec["verdict"] == "FEASIBLE" and not rec["phase1_used"]:
        errs = {k: _rel(getattr(r, k), rec[k]) for k in ("psi", "phi", "margin")}
        assert max(errs.values()) <= 1e-6, errs
        assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
        assert abs(r.iterations - rec["iterations"]) <= its, (r.iterations, rec["iterations"])
    return errs


def _perm(g, n, L0):
    pairs = g.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_n100_vs_oracle(P, prec):
    recs = [r for r in _large() if r["tag"] == "n100" and r["seed"] == 0]
    if not recs:
        pytest.skip("no stored oracle end point of the n = 100 system")
    sy = W.c2_system(0)
    print(f"n100 {prec}", flush=True)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, precision=prec)
    errs = _check(recs[0], r, its=1 if prec == "fp64" else 2)
    print(f"n100 {prec}: verdict {r.verdict_name}, {r.iterations} iterations "
          f"({r.iters_lowprec} with {prec} assembly, {r.ir_steps} refinement steps), "
          f"relative error vs the FP64 oracle: " + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()),
          flush=True)
    if prec != "fp64":
        assert r.iters_lowprec >= 1


def test_n32_heldout_vs_oracle(P):
    recs = {r["seed"]: r for r in _large() if r["tag"] == "n32"}
    if not recs:
        pytest.skip("no stored oracle end points of the n = 32 family")
    seeds = sorted(recs)
    sys_ = [W.warm_system(s) for s in seeds]
    print(f"n32 held-out batch of {len(seeds)}", flush=True)
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    for prec in ("fp64", "fp32"):
        rs = P.ipm_solve_batched(gs, precision=prec)
        for s, r in zip(seeds, rs):
            _check(recs[s], r, its=1 if prec == "fp64" else 2)


def test_mixed_largest_members_vs_oracle(P):
    recs = [r for r in _large() if r["tag"].startswith("mixed")]
    if not recs:
        pytest.skip("no stored oracle end points of large mixed-batch members")
    mixed = W.mixed_systems(512)
    idx = [r["index"] for r in recs]
    print(f"mixed members {idx}", flush=True)
    gs = [P.polya_setup(mixed[i].A, mixed[i].n, mixed[i].l, mixed[i].dp, mixed[i].d) for i in idx]
    for prec in ("fp64", "fp32"):
        rs = P.ipm_solve_batched(gs, precision=prec)
        for rec, r in zip(recs, rs):
            _check(rec, r, its=1 if prec == "fp64" else 2)


def test_whole_mixed_batch(P):
    """The batched form's own configuration: all 512 members in one solve
    with FP32 assembly."""
    mixed = W.mixed_systems(512)
    gold = _small_mixed()
    gold.update({r["index"]: r for r in _large() if r["tag"].startswith("mixed")})
    print(f"mixed batch of 512 ({len(gold)} with oracle end points)", flush=True)
    gs = P.polya_setup_batched([(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in mixed])
    rs = P.ipm_solve_batched(gs, precision="fp32")
    print("solved; checking", flush=True)
    for i, r in enumerate(rs):
        if i in gold:
            _check(gold[i], r, its=2)
        assert r.verdict_name in ("FEASIBLE", "INFEASIBLE", "UNKNOWN")
        if r.verdict_name == "FEASIBLE" and not r.phase1_used:
            assert abs(float(np.sum(r.y)) - r.psi) <= 1e-9 * abs(r.psi)
    # the certificate's blocks through the oracle's operators on a spread
    # sample (every 32nd member and the largest one)
    Ks = [comb(sy.l + sy.dp - 1, sy.dp) * sy.n * (sy.n + 1) // 2 for sy in mixed]
    sample = sorted(set(range(0, 512, 32)) | {int(np.argmax(Ks))})
    for i in sample:
        sy, g, r = mixed[i], gs[i], rs[i]
        if r.verdict_name != "FEASIBLE":
            continue
        sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
        y = np.empty_like(r.y)
        y[_perm(g, sy.n, sdp.L0)] = r.y
        Q = sdp.BT(y)
        lam = np.array([np.linalg.eigvalsh(Q[j])[0] for j in range(sdp.nb)])
        assert lam.min() > 0
        assert abs(r.margin - float(np.min(lam / sdp.scale))) <= 1e-6 * abs(r.margin)
    counts = {}
    for r in rs:
        counts[r.verdict_name] = counts.get(r.verdict_name, 0) + 1
    print(f"verdicts {counts}", flush=True)

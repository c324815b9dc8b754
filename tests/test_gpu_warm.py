"""Warm-started IPM on the GPU against the oracle's warm start (marker: gpu).

The starting data (y, log block scales of X) are the oracle's own iterate
after k cold iterations, so the inputs come from oracle/ only.  Both sides
project them into the interior the same way (the oracle with the symmetric
eigensolver, the library with bisection on Cholesky) and must reach the same
verdict and objective; rejected warm starts must give the cold answer.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import ipm, sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _perm(g, n, L0):
    pairs = g.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


CASES = [("plain", 0, 8), ("plain", 3, 12), ("plain", 7, 16), ("n10", 1, 12), ("n10", 5, 16)]


@pytest.mark.parametrize("tag,seed,k", CASES)
def test_warm_start_parity(P, tag, seed, k):
    sy = W.plain_system(seed) if tag == "plain" else W.c1_system(seed)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    mid = ipm.ipm_run(ipm.PaperOps(sdp), ipm.Options(), max_iter=k)
    logx = np.log(np.trace(mid.X, axis1=1, axis2=2) / sy.n)
    want = ipm.ipm_solve(sdp, warm=(mid.y, logx))
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    perm = _perm(g, sy.n, sdp.L0)
    print(f"warm {tag} seed={seed} k={k}", flush=True)
    r = P.ipm_solve(g, warm_y=mid.y[perm], warm_logx=logx)
    assert r.warm_used == want.warm_used and r.warm_fallback == want.warm_fallback
    assert r.verdict_name == ipm.VERDICT_NAMES[want.verdict]
    assert abs(r.psi - want.psi) <= 1e-6 * abs(want.psi)
    assert abs(r.margin - want.margin) <= 1e-6 * abs(want.margin)
    assert abs(r.iterations - want.iterations) <= 1, (r.iterations, want.iterations)
    assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8


def test_rejected_warm_start_gives_cold_answer(P):
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        recs = [r for r in json.load(fh) if r["tag"] == "n10"][:6]
    sys_ = [W.c1_system(r["seed"]) for r in recs]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    rng = np.random.default_rng(7)
    wy = [rng.standard_normal(g.K) for g in gs]
    print("rejected warm starts", flush=True)
    rs = P.ipm_solve_batched(gs, warm_y=wy, warm_iter_cap=2)
    cold = P.ipm_solve_batched(gs)
    for rec, r, c in zip(recs, rs, cold):
        assert r.warm_fallback and not r.warm_used and r.warm_iterations == 2
        assert r.verdict_name == rec["verdict"]
        assert r.iterations == c.iterations and np.array_equal(r.y, c.y)


def test_label_capture_matches_trajectory(P):
    """label_gap records the iterate of the first iteration with gap <= the
    threshold: warm-starting from it follows the same end point."""
    sy = W.c1_system(2)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, label_gap=1e-2, record_history=1)
    assert r.label_iter > 0
    h = {e["iter"]: e for e in r.history}
    assert h[r.label_iter]["gap_rel"] <= 1e-2 < h[r.label_iter - 1]["gap_rel"]
    w = P.ipm_solve(g, warm_y=r.label_y, warm_logx=r.label_logx)
    assert w.warm_used and w.verdict == P.FEASIBLE
    assert abs(w.psi - r.psi) <= 1e-6 * abs(r.psi)
    assert w.iterations < r.iterations

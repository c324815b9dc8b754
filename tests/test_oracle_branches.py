"""Pins of the oracle's less-travelled branches, each against something other
than the oracle itself:

* the Schur factorisation's diagonal shift (Alg. 2 root step 1 with the
  failure policy of the design notes): on a matrix built with a known
  negative eigenvalue the first shift that succeeds is predictable from the
  spectrum, and a definite matrix is never shifted unless forced;
* the refinement of a shifted solve converges to the solution of the
  UNSHIFTED matrix at the rate (tau ||Lam^-1||)^(steps+1);
* the phase-I margin SDP and its rescaled certificate: for A_i = -aI the
  normalised margin t* and the rescaled certificate's objective have closed
  forms that follow from the paper's own optimum by homogeneity;
* the paper-literal set-up (derivative blocks C_j = 0, eq. Cj as printed) and
  the paper's absolute gap test (Section IV-A);
* Mehrotra's sigma reaches the same optimum as the fixed sigma.
"""
import numpy as np
import pytest

from oracle import ipm, sdp as S
from paper_1411_3769_amd import workloads as W


def _spd_with_spectrum(ev, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((len(ev), len(ev))))
    M = (Q * np.asarray(ev)) @ Q.T
    return 0.5 * (M + M.T)


def test_shift_first_success_from_spectrum():
    """lambda_min = -3e-12 * lambda_max: shifts 1e-14 and 1e-12 (x max diag)
    leave it negative, 1e-10 makes it positive with a wide margin, so the
    factorisation must succeed exactly at the third level."""
    ev = np.concatenate([np.linspace(1.0, 2.0, 47), [1e-3, 1e-6, -3e-12 * 2.0]])
    Lam = _spd_with_spectrum(ev, 0)
    dmax = float(np.max(np.diag(Lam)))
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(Lam)
    R, tau = ipm._factor_with_shift(Lam, ipm.Options())
    assert R is not None
    assert abs(tau / dmax - 1e-10) <= 1e-10 * 1e-12   # 1e-14 * 100 * 100, to rounding
    assert np.abs(R @ R.T - (Lam + tau * np.eye(len(ev)))).max() <= 1e-13 * dmax


def test_shift_never_for_definite_unless_forced():
    Lam = _spd_with_spectrum(np.linspace(1.0, 10.0, 30), 1)
    R, tau = ipm._factor_with_shift(Lam, ipm.Options())
    assert tau == 0.0
    dmax = float(np.max(np.diag(Lam)))
    R, tau = ipm._factor_with_shift(Lam, ipm.Options(shift_force=1e-9))
    assert abs(tau - 1e-9 * dmax) <= 1e-24 * dmax
    assert np.abs(R @ R.T - (Lam + tau * np.eye(30))).max() <= 1e-13 * dmax


def test_shift_gives_up_beyond_cap():
    """lambda_min = -1e-3 lambda_max is beyond the largest shift 1e-6."""
    ev = np.concatenate([np.linspace(1.0, 2.0, 20), [-2e-3]])
    R, tau = ipm._factor_with_shift(_spd_with_spectrum(ev, 2), ipm.Options())
    assert R is None and tau is None


@pytest.mark.parametrize("steps", [0, 1, 2, 3])
def test_refinement_converges_to_unshifted_solution(steps):
    """kappa = tau ||Lam^-1|| = 1e-2: the shifted solve is off by about kappa,
    each refinement step against the unshifted matrix multiplies the error by
    about kappa.  Refining against the shifted matrix would stall at kappa."""
    K = 40
    ev = np.geomspace(1e-4, 1.0, K)
    Lam = _spd_with_spectrum(ev, 3)
    tau = 1e-6
    kappa = tau / 1e-4
    R = np.linalg.cholesky(Lam + tau * np.eye(K))
    rhs = np.random.default_rng(4).standard_normal(K)
    want = np.linalg.solve(Lam, rhs)
    x = ipm._solve(R, tau, Lam, rhs, ipm.Options(ir_steps=steps))
    err = np.linalg.norm(x - want) / np.linalg.norm(want)
    assert err <= 1.5 * kappa ** (steps + 1)
    if steps == 0:
        assert err >= 0.2 * kappa


@pytest.mark.parametrize("a", [0.2, 2.0])
@pytest.mark.parametrize("l,dp,d", [(2, 1, 1), (3, 1, 1), (3, 2, 1)])
def test_phase1_closed_form_and_rescaled_certificate(a, l, dp, d):
    """A_i = -aI with delta = eps = theta: the paper's optimum is
    v* = l^dp n theta max(1, 1/(2a)); by homogeneity the phase-I optimum is
    t* = theta / v*, and the phase-I solution rescaled by theta / t* is a
    paper optimum with objective v* and margin theta."""
    n = 3
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    sdp = S.make_sdp(A, n, l, dp, d)
    r = ipm.ipm_solve(sdp, ipm.Options(verdict_mode="phase1_only"))
    v_star = l ** dp * n * 1e-3 * max(1.0, 1.0 / (2 * a))
    assert r.phase1_used and r.verdict == ipm.FEASIBLE
    assert abs(r.t_star - 1e-3 / v_star) <= 1e-6 * (1e-3 / v_star)
    assert abs(r.psi - v_star) <= 1e-6 * v_star
    assert abs(r.margin - 1e-3) <= 1e-6 * 1e-3


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_phase1_only_plain_seeds(seed):
    """Plain seeds through phase-I: FEASIBLE, t* > 0, the rescaled certificate
    is tight at the margin delta (some block attains the phase-I optimum),
    and its objective is no better than the paper's optimum (it is a
    feasible point of the paper's SDP)."""
    sy = W.plain_system(seed)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r1 = ipm.ipm_solve(sdp, ipm.Options(verdict_mode="phase1_only"))
    r0 = ipm.ipm_solve(sdp)
    assert r1.verdict == ipm.FEASIBLE and r1.t_star > 0
    assert abs(r1.margin - 1e-3) <= 1e-6 * 1e-3
    assert r1.psi >= r0.psi * (1 - 1e-7)
    ok, mg, _, _ = ipm.certificate(sdp, r1.y)
    assert ok and mg >= 1e-3 * (1 - 1e-6)


def test_phase1_only_twin_infeasible():
    sy = W.plain_system(0, twin=True)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = ipm.ipm_solve(sdp, ipm.Options(verdict_mode="phase1_only"))
    assert r.verdict == ipm.INFEASIBLE and r.t_star < -1e-6


@pytest.mark.parametrize("a", [0.2, 2.0])
def test_paper_literal_closed_form(a):
    """Derivative blocks with C_j = 0 (eq. Cj as printed): the optimum of
    A_i = -aI becomes l^dp n delta (the derivative LMIs no longer bind)."""
    n, l, dp, d = 3, 3, 1, 1
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    sdp = S.make_sdp(A, n, l, dp, d, paper_literal=True)
    assert np.all(sdp.cdiag[sdp.L:] == 0.0)
    r = ipm.ipm_solve(sdp)
    want = l ** dp * n * 1e-3
    assert r.verdict == ipm.FEASIBLE
    assert abs(r.psi - want) <= 1e-6 * want


def test_absolute_gap_rule():
    """The paper's stopping test |a^T y - tr(CX)| <= 1e-8 alone: at exit the
    absolute gap meets it, the objective is within it (plus the residual
    slack) of the closed-form optimum, and it stops no later than the
    scale-relative rule."""
    n, l, dp, d, a = 3, 3, 1, 1, 2.0
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    sdp = S.make_sdp(A, n, l, dp, d, paper_literal=True)
    want = l ** dp * n * 1e-3
    r = ipm.ipm_solve(sdp, ipm.Options(stop_rule="absolute"))
    r0 = ipm.ipm_solve(sdp)
    assert r.verdict == ipm.FEASIBLE
    assert r.gap_abs <= 1e-8
    assert abs(r.psi - want) <= 1e-8 + 1e-6 * want
    assert r.iterations <= r0.iterations


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mehrotra_same_optimum(seed):
    sy = W.plain_system(seed)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r0 = ipm.ipm_solve(sdp)
    r1 = ipm.ipm_solve(sdp, ipm.Options(sigma_rule="mehrotra"))
    assert r1.verdict == r0.verdict == ipm.FEASIBLE
    assert abs(r1.psi - r0.psi) <= 1e-6 * abs(r0.psi)
    assert abs(r1.margin - r0.margin) <= 1e-6 * abs(r0.margin)
    assert r1.iterations <= r0.iterations


@pytest.mark.parametrize("a", [0.2, 2.0])
def test_mehrotra_closed_form(a):
    n, l, dp, d = 3, 2, 1, 2
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    r = ipm.ipm_solve(S.make_sdp(A, n, l, dp, d), ipm.Options(sigma_rule="mehrotra"))
    want = l ** dp * n * max(1e-3, 1e-3 / (2 * a))
    assert r.verdict == ipm.FEASIBLE and abs(r.psi - want) <= 1e-6 * want


@pytest.mark.parametrize("force", [1e-12, 1e-8])
def test_forced_shift_keeps_end_point(force):
    """Every factorisation shifted, then refined against the unshifted
    matrix: the end point is that of the unshifted run."""
    sy = W.plain_system(1)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r0 = ipm.ipm_solve(sdp)
    r1 = ipm.ipm_solve(sdp, ipm.Options(shift_force=force))
    assert r1.verdict == r0.verdict == ipm.FEASIBLE
    assert r1.chol_shifts == r1.iterations and r0.chol_shifts == 0
    # both runs meet the 1e-8 relative gap test around the same optimum
    assert abs(r1.psi - r0.psi) <= 2e-8 * abs(r0.psi)
    assert abs(r1.iterations - r0.iterations) <= 1

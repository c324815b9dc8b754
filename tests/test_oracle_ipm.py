"""Pins of the oracle's interior-point solver against closed forms and
invariants: the scalar (n=1) case is a linear programme whose verdict is
known; with all vertices equal the optimum follows from the Lyapunov equation
(l=1 included); A = -aI has an explicit optimum; the infeasible twin can have no
certificate; Theorem 3 on a dense solver; KKT residuals; certificate soundness
on the simplex."""
import numpy as np
import pytest
from scipy.linalg import solve_continuous_lyapunov

from oracle import ipm, polya, sdp as S
from paper_1411_3769_amd import workloads as W

OPT = ipm.Options()
Wmat = lambda n: 0.5 * (np.eye(n) + np.ones((n, n)))


def _solve(A, n, l, dp, d, **kw):
    sdp = S.make_sdp(A, n, l, dp, d, **kw)
    return sdp, ipm.ipm_solve(sdp, OPT)


@pytest.mark.parametrize("l,dp,d", [(1, 1, 1), (2, 1, 1), (3, 2, 1), (3, 1, 2)])
def test_scalar_case_verdicts(l, dp, d):
    """n = 1: FEASIBLE iff every vertex is negative, for any dp and d."""
    rng = np.random.default_rng(l * 10 + dp)
    neg = -rng.uniform(0.2, 2.0, size=(l, 1, 1))
    _, r = _solve(neg, 1, l, dp, d)
    assert r.verdict == ipm.FEASIBLE
    pos = neg.copy()
    pos[l - 1] = 0.5
    _, r = _solve(pos, 1, l, dp, d)
    assert r.verdict == ipm.INFEASIBLE


@pytest.mark.parametrize("a", [0.2, 2.0])
@pytest.mark.parametrize("l,dp,d", [(1, 1, 1), (2, 1, 2), (3, 2, 1)])
def test_scaled_identity_closed_form(a, l, dp, d):
    """A_i = -a I: optimum l^dp * n * max(delta, eps/(2a))."""
    n = 3
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    sdp, r = _solve(A, n, l, dp, d)
    want = l ** dp * n * max(1e-3, 1e-3 / (2 * a))
    assert r.verdict == ipm.FEASIBLE
    assert abs(r.psi - want) <= 1e-6 * want
    assert abs(r.phi - want) <= 1e-6 * want


@pytest.mark.parametrize("l,dp,d", [(1, 1, 1), (1, 2, 2), (2, 1, 1), (2, 2, 1), (3, 1, 2)])
def test_equal_vertices_lyapunov(l, dp, d):
    """All vertices equal to a Hurwitz A: the optimum is
    l^dp * eps * <P_lyap, (I + 11^T)/2> with A^T P_lyap + P_lyap A = -I,
    provided eps * lambda_min(P_lyap) >= delta (l = 1 is the plain Lyapunov
    inequality)."""
    n = 3
    rng = np.random.default_rng(42 + l + dp)
    G = rng.standard_normal((n, n))
    A0 = G - (np.max(np.linalg.eigvals(G).real) + 0.7) * np.eye(n)
    P_lyap = solve_continuous_lyapunov(A0.T, -np.eye(n))
    eps = 1e-3
    delta = 0.5 * eps * np.linalg.eigvalsh(P_lyap)[0]
    A = np.repeat(A0[None], l, axis=0)
    sdp, r = _solve(A, n, l, dp, d, delta=delta, eps=eps)
    want = l ** dp * eps * np.sum(P_lyap * Wmat(n))
    assert r.verdict == ipm.FEASIBLE
    assert abs(r.psi - want) <= 1e-6 * want
    # every coefficient of the optimal P is eps * P_lyap times the multinomial dp!/h!
    for hi, h in enumerate(polya.monomials(l, dp)):
        ref = eps * P_lyap * polya.multinomial(dp, h)
        assert np.abs(r.P[hi] - ref).max() <= 1e-4 * np.abs(ref).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_plain_seed_and_twin(seed):
    sy = W.plain_system(seed)
    sdp, r = _solve(sy.A, sy.n, sy.l, sy.dp, sy.d)
    assert r.verdict == ipm.FEASIBLE
    assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
    tw = W.plain_system(seed, twin=True)
    # the twin's first vertex has max Re eig = +1: no certificate at any degree
    assert np.max(np.linalg.eigvals(tw.A[0]).real) == pytest.approx(1.0)
    _, r2 = _solve(tw.A, tw.n, tw.l, tw.dp, tw.d)
    assert r2.verdict == ipm.INFEASIBLE
    assert r2.phase1_used and r2.t_star < -1e-6


def test_kkt_at_exit():
    sy = W.plain_system(4)
    sdp = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    run = ipm.ipm_run(ipm.PaperOps(sdp), OPT)
    assert run.reason == ipm.CONVERGED
    a = sdp.a()
    assert np.linalg.norm(sdp.B(run.X) - a) <= 1e-8 * (1 + np.linalg.norm(a))
    Zc = sdp.BT(run.y) - sdp.C_blocks()
    assert np.linalg.norm(Zc - run.Z) <= 1e-8 * (1 + np.linalg.norm(sdp.C_blocks()))
    assert all(ipm.chol_ok(x) for x in run.X) and all(ipm.chol_ok(z) for z in run.Z)
    # complementarity: tr(ZX) equals the duality gap psi - phi for a feasible pair
    trZX = sum(np.trace(run.Z[j] @ run.X[j]) for j in range(sdp.nb))
    assert abs(trZX - (run.psi - run.phi)) <= 1e-9 * abs(run.psi)
    assert trZX <= 1e-7 * abs(run.psi)


def test_certificate_soundness_on_simplex():
    sy = W.plain_system(0)
    sdp, r = _solve(sy.A, sy.n, sy.l, sy.dp, sy.d)
    assert r.verdict == ipm.FEASIBLE and r.margin > 0
    Wp = polya.monomials(sy.l, sy.dp)
    rng = np.random.default_rng(9)
    pts = [np.array(g, float) / 4 for g in polya.monomials(sy.l, 4)]
    pts += list(rng.dirichlet(np.ones(sy.l), size=2000))
    for a in pts:
        Pa = sum(r.P[i] * np.prod(a ** np.array(h)) for i, h in enumerate(Wp))
        Aa = np.tensordot(a, sy.A, axes=1)
        assert np.linalg.eigvalsh(Pa)[0] > 0
        assert np.linalg.eigvalsh(Aa.T @ Pa + Pa @ Aa)[-1] < 0
        assert np.max(np.linalg.eigvals(Aa).real) < 0


def test_theorem3_dense_solver():
    """Started from block-diagonal X, Z the dense solver's iterates stay
    block-diagonal (off-block entries exactly zero) and reach the same
    objective as the block solver."""
    rng = np.random.default_rng(3)
    n, l = 2, 2
    A = rng.standard_normal((l, n, n)) - 2.5 * np.eye(n)
    sdp = S.make_sdp(A, n, l, 1, 1)
    Xd, Zd, yd, hist = ipm.dense_ipm(sdp, OPT, iters=60)
    mask = S.blockdiag(np.ones((sdp.nb, n, n))) == 0
    assert np.all(Xd[mask] == 0.0) and np.all(Zd[mask] == 0.0)
    r = ipm.ipm_solve(sdp, OPT)
    assert r.verdict == ipm.FEASIBLE
    assert abs(hist[-1]["psi"] - r.psi) <= 1e-6 * abs(r.psi)


def test_phase1_schur_matches_definition():
    sdp = S.make_sdp(np.random.default_rng(2).standard_normal((2, 2, 2)), 2, 2, 1, 1)
    p1 = ipm.Phase1Ops(sdp)
    X = W.random_spd_blocks(3, sdp.nb, 2)
    Zi = np.linalg.inv(W.random_spd_blocks(4, sdp.nb, 2))
    ref = np.empty((sdp.K, sdp.K))
    for l in range(sdp.K):
        e = np.zeros(sdp.K)
        e[l] = 1.0
        ref[:, l] = p1.B(np.einsum("jab,jbc,jcd->jad", Zi, p1.BT(e), X))
    assert np.abs(p1.schur(X, Zi) - ref).max() <= 1e-12 * np.abs(ref).max()
    # phase-I operators are adjoint as well
    y = np.random.default_rng(5).standard_normal(sdp.K)
    Wb = np.random.default_rng(6).standard_normal((sdp.nb, 2, 2))
    assert np.isclose(y @ p1.B(Wb), sum(np.trace(Wb[j] @ p1.BT(y)[j]) for j in range(sdp.nb)))


def test_ladder_keeps_blocks_pd():
    rng = np.random.default_rng(8)
    V = W.random_spd_blocks(1, 6, 4)
    dV = rng.standard_normal((6, 4, 4))
    dV = dV + dV.transpose(0, 2, 1)
    t = ipm.ladder(V, dV, OPT)
    assert t is not None and 0 < t <= 1
    assert all(ipm.chol_ok(V[j] + t * dV[j]) for j in range(6))
    assert ipm.ladder(V, np.zeros_like(dV), OPT) == 1.0


@pytest.mark.slow
def test_n10_seed_feasible():
    sy = W.c1_system(0)
    sdp, r = _solve(sy.A, sy.n, sy.l, sy.dp, sy.d)
    assert r.verdict == ipm.FEASIBLE
    assert r.margin == pytest.approx(1e-3, rel=1e-6)

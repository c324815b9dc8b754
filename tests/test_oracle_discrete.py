"""Pins of the oracle's discrete-time form (oracle/discrete.py: the
generalized LMI of Section III-C instantiated for x+ = A(alpha) x):

* the closed form of the scalar case with equal vertices: the optimum is
  max(delta, eps / (1 - |a|)) for |a| < 1, and |a| > 1 is refuted;
* the Polya coefficients as a polynomial identity: sum_gamma alpha^gamma
  M_gamma(y) equals (sum alpha)^d2 [[(sum alpha)^da P, P A], [A^T P,
  (sum alpha)^da P]] at random simplex points (signs, b, H and the block
  layout);
* B, B^T against B_k materialised from the definition, and the Schur
  complement by definition against the dense brute force;
* verdicts: a contractive polytope is certified and its P(alpha) checks out
  pointwise (P > 0, A^T P A - P < 0 on a simplex grid); a vertex with
  spectral radius above 1 is never certified; a Hurwitz-but-not-Schur system
  and a Schur-but-not-Hurwitz one separate the two forms.
"""
import numpy as np
import pytest

from oracle import discrete as D, ipm, polya, sdp as S


@pytest.mark.parametrize("a", [0.5, -0.7, 0.9])
@pytest.mark.parametrize("d", [1, 2])
def test_scalar_closed_form(a, d):
    s = D.make_discrete_sdp(np.full((3, 1, 1), a), 1, 3, 0, d)
    r = ipm.ipm_solve(s)
    assert r.verdict == ipm.FEASIBLE
    want = max(1e-3, 1e-3 / (1 - abs(a)))
    assert abs(r.psi - want) <= 1e-6 * want


@pytest.mark.parametrize("a", [1.2, -1.05])
def test_scalar_unstable_refuted(a):
    r = ipm.ipm_solve(D.make_discrete_sdp(np.full((3, 1, 1), a), 1, 3, 0, 1))
    assert r.verdict == ipm.INFEASIBLE


def _poly(coefs, exps, alpha):
    return sum(c * np.prod(alpha ** np.array(e)) for c, e in zip(coefs, exps))


@pytest.mark.parametrize("n,l,dp,da,d", [(2, 3, 1, 1, 1), (2, 2, 2, 1, 2), (3, 3, 1, 2, 1), (1, 4, 2, 1, 0)])
def test_coefficients_polynomial_identity(n, l, dp, da, d):
    rng = np.random.default_rng(n + 10 * l + 100 * dp + 1000 * da + d)
    Wa = polya.monomials(l, da)
    A = rng.standard_normal((len(Wa), n, n))
    s = D.make_discrete_sdp(A, n, l, dp, d, da=da)
    y = rng.standard_normal(s.K)
    M = s.M_of_y(y)
    P = s.P_of_y(y)
    Wp, WM = polya.monomials(l, dp), polya.monomials(l, dp + da + d)
    for alpha in rng.dirichlet(np.ones(l), size=5):
        Pa, Aa, sa = _poly(P, Wp, alpha), _poly(A, Wa, alpha), alpha.sum()
        want = np.block([[sa ** da * Pa, Pa @ Aa], [Aa.T @ Pa, sa ** da * Pa]]) * sa ** d
        got = _poly(M, WM, alpha)
        assert np.abs(got - want).max() <= 1e-12 * (1 + np.abs(want).max())


def test_operators_against_dense_definition():
    rng = np.random.default_rng(7)
    s = D.make_discrete_sdp(rng.standard_normal((3, 2, 2)), 2, 3, 1, 1)
    y = rng.standard_normal(s.K)
    dense = sum(y[k] * s.dense_B(k) for k in range(s.K))
    assert np.abs(dense - S.blockdiag(s.BT(y))).max() <= 1e-12 * np.abs(dense).max()
    W = rng.standard_normal((s.nb, 4, 4))
    Wd = S.blockdiag(W)
    want = np.array([np.trace(s.dense_B(k) @ Wd) for k in range(s.K)])
    assert np.abs(s.B(W) - want).max() <= 1e-12 * np.abs(want).max()


def test_schur_definition_against_dense():
    rng = np.random.default_rng(8)
    s = D.make_discrete_sdp(rng.standard_normal((2, 2, 2)), 2, 2, 1, 1)
    def spd(k):
        G = rng.standard_normal((k, 4, 4))
        return G @ G.transpose(0, 2, 1) + 4 * np.eye(4)
    X, Zi = spd(s.nb), np.linalg.inv(spd(s.nb))
    want = S.schur_dense(s, X, Zi)
    got = s.schur(X, Zi)
    assert np.abs(got - want).max() <= 1e-11 * np.abs(want).max()


def _contractive(rng, l, n, rho):
    out = []
    for _ in range(l):
        Q = rng.standard_normal((n, n))
        out.append(rho * Q / np.linalg.norm(Q, 2))
    return np.stack(out)


@pytest.mark.parametrize("seed", [0, 1])
def test_contractive_polytope_certified(seed):
    rng = np.random.default_rng(seed)
    l, n = 3, 3
    A = _contractive(rng, l, n, 0.9)
    s = D.make_discrete_sdp(A, n, l, 1, 1)
    r = ipm.ipm_solve(s)
    assert r.verdict == ipm.FEASIBLE
    Wp = polya.monomials(l, 1)
    grid = [np.array(m, dtype=float) / 12 for m in polya.monomials(l, 12)]
    lo, hi = D.lyapunov_margin(lambda a: np.tensordot(a, A, 1), lambda a: _poly(r.P, Wp, a), grid)
    assert lo > 0 and hi < 0


@pytest.mark.parametrize("dp,d", [(0, 1), (1, 2)])
def test_unstable_vertex_never_certified(dp, d):
    rng = np.random.default_rng(3)
    A = _contractive(rng, 3, 2, 0.5)
    A[1] = np.array([[1.1, 0.3], [0.0, 0.2]])     # spectral radius 1.1
    r = ipm.ipm_solve(D.make_discrete_sdp(A, 2, 3, dp, d))
    assert r.verdict != ipm.FEASIBLE


def test_forms_separate():
    """-2I is Hurwitz (spectral radius 2); 0.5 I is Schur (eigenvalues > 0)."""
    hur = np.stack([-2.0 * np.eye(2), -2.0 * np.eye(2) + [[0, 0.1], [0, 0]]])
    sch = np.stack([0.5 * np.eye(2), 0.5 * np.eye(2) + [[0, 0.1], [0, 0]]])
    assert ipm.ipm_solve(S.make_sdp(hur, 2, 2, 0, 1)).verdict == ipm.FEASIBLE
    assert ipm.ipm_solve(D.make_discrete_sdp(hur, 2, 2, 0, 1)).verdict != ipm.FEASIBLE
    assert ipm.ipm_solve(S.make_sdp(sch, 2, 2, 0, 1)).verdict != ipm.FEASIBLE
    assert ipm.ipm_solve(D.make_discrete_sdp(sch, 2, 2, 0, 1)).verdict == ipm.FEASIBLE

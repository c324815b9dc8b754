"""Pins of the oracle's SDP operators and Schur complement against the dense
materialisation of eq. Ai/Aij (brute force on tiny inputs), adjointness and
structural properties."""
import numpy as np
import pytest

from oracle import sdp as S
from paper_1411_3769_amd import workloads as W


def _rand_sdp(n, l, dp, d, seed=0):
    A = np.random.default_rng(seed).standard_normal((l, n, n))
    return S.make_sdp(A, n, l, dp, d)


CASES = [(2, 2, 1, 1), (3, 3, 1, 1), (2, 3, 2, 1), (3, 2, 1, 2), (1, 3, 2, 2)]


@pytest.mark.parametrize("n,l,dp,d", CASES)
def test_operators_match_dense(n, l, dp, d):
    sdp = _rand_sdp(n, l, dp, d)
    rng = np.random.default_rng(3)
    y = rng.standard_normal(sdp.K)
    Wb = rng.standard_normal((sdp.nb, n, n))       # not symmetric on purpose
    dense = [sdp.dense_B(k) for k in range(sdp.K)]
    Wd = S.blockdiag(Wb)
    assert np.allclose([np.trace(Bk @ Wd) for Bk in dense], sdp.B(Wb), rtol=0, atol=1e-12)
    assert np.allclose(sum(y[k] * dense[k] for k in range(sdp.K)), S.blockdiag(sdp.BT(y)),
                       rtol=0, atol=1e-12)
    for Bk in dense:
        assert np.array_equal(Bk, Bk.T)
    # adjointness y^T B(W) = sum_j tr(W_j B^T(y)_j)
    lhs = y @ sdp.B(Wb)
    rhs = sum(np.trace(Wb[j] @ sdp.BT(y)[j]) for j in range(sdp.nb))
    assert abs(lhs - rhs) <= 1e-12 * (1 + abs(lhs))


def test_basis_and_objective():
    for n in (1, 2, 5, 7):
        pairs = S.basis_pairs(n)
        assert len(pairs) == n * (n + 1) // 2
        assert sorted(pairs) == sorted((p, q) for p in range(n) for q in range(p, n))
    sdp = _rand_sdp(4, 3, 2, 1)
    rng = np.random.default_rng(5)
    P = np.array([(lambda M: M + M.T)(rng.standard_normal((4, 4))) for _ in range(sdp.L0)])
    y = sdp.y_of_P(P)
    assert np.array_equal(sdp.P_of_y(y), P)
    # a^T y is the sum of the upper-triangular entries of all P_h (eq. a)
    assert np.isclose(sdp.a() @ y, sum(np.triu(Ph).sum() for Ph in P))
    # ... which equals <sum_h P_h, (I + 11^T)/2>
    Wm = 0.5 * (np.eye(4) + np.ones((4, 4)))
    assert np.isclose(sdp.a() @ y, np.sum(P.sum(0) * Wm))


@pytest.mark.parametrize("n,l,dp,d", CASES[:4])
def test_schur_three_ways(n, l, dp, d):
    sdp = _rand_sdp(n, l, dp, d, seed=11)
    X = W.random_spd_blocks(1, sdp.nb, n)
    Zi = np.linalg.inv(W.random_spd_blocks(2, sdp.nb, n))
    Ld = S.schur_dense(sdp, X, Zi)
    Lf = S.schur_definition(sdp, X, Zi)
    Le = S.schur_expanded(sdp, X, Zi)
    scale = np.abs(Ld).max()
    assert np.abs(Lf - Ld).max() <= 1e-13 * scale
    assert np.abs(Le - Ld).max() <= 1e-13 * scale
    assert np.allclose(Le, Le.T, rtol=0, atol=1e-13 * scale)
    assert np.linalg.eigvalsh(Le)[0] > 0          # PD for PD iterates (B_k independent)


def test_schur_expanded_vs_definition_medium():
    sy = W.c1_system(3)
    sdp = S.make_sdp(sy.A[:, :4, :4], 4, 4, 2, 2)
    X = W.random_spd_blocks(5, sdp.nb, 4)
    Zi = np.linalg.inv(W.random_spd_blocks(6, sdp.nb, 4))
    Le = S.schur_expanded(sdp, X, Zi)
    Lf = S.schur_definition(sdp, X, Zi)
    assert np.abs(Le - Lf).max() <= 1e-12 * np.abs(Lf).max()


def test_theorem3_block_structure_of_operators():
    # B^T maps into the block-diagonal subspace S_{L,M,n} (used in Theorem 3)
    sdp = _rand_sdp(3, 3, 1, 1)
    y = np.random.default_rng(0).standard_normal(sdp.K)
    Dn = sum(y[k] * sdp.dense_B(k) for k in range(sdp.K))
    mask = S.blockdiag(np.ones((sdp.nb, 3, 3))) == 0
    assert np.all(Dn[mask] == 0.0)

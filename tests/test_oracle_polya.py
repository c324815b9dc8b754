"""Pins of the oracle's exact Polya set-up against facts the paper and the
mathematics fix: printed worked examples, closed forms, brute-force expansion,
coefficient sums and polynomial identities at random points of the simplex."""
import itertools
from math import comb, factorial

import numpy as np
import pytest

from conftest import read_golden
from oracle import polya
from oracle.sdp import make_sdp


GRID = [(l, dp, d) for l in (1, 2, 3, 4) for dp in (0, 1, 2) for d in (0, 1, 2, 3)]


def test_counts_match_enumeration():
    for l in range(1, 6):
        for d in range(0, 6):
            assert polya.f(l, d) == len(polya.monomials(l, d))
            assert len(set(polya.monomials(l, d))) == polya.f(l, d)
    assert polya.f(0, 3) == 0


@pytest.mark.parametrize("n,l,dp,d,L0,L,M,K", [
    (4, 3, 1, 1, 3, 6, 10, 30),            # plain case: 6 P-blocks, 10 derivative blocks
    (10, 4, 2, 2, 10, 35, 56, 550),        # n=10 family
    (100, 4, 1, 3, 4, 35, 56, 20200),      # n=100 family
    (32, 4, 1, 2, 4, 20, 35, 2112),        # warm-start family
    (48, 5, 2, 4, 15, 210, 330, 17640),    # largest mixed-batch shape
])
def test_problem_dimensions(n, l, dp, d, L0, L, M, K):
    c = polya.counts(l, dp, 1, d, d, n)
    assert (c["L0"], c["L"], c["M"], c["K"]) == (L0, L, M, K)


def test_paper_example_dimensions():
    # Example 3: K = 50/90/224 and X of size 200/385/1092 with d1 = d2 = 1
    # are reproduced by dp = 1 at (n, l) = (4,5), (5,6), (7,8).
    for (n, l, K, m) in [(4, 5, 50, 200), (5, 6, 90, 385), (7, 8, 224, 1092)]:
        c = polya.counts(l, 1, 1, 1, 1, n)
        assert c["K"] == K and c["m"] == m
    # Fig. 4 caption: l=10, dp=2, da=3, d1=d2=4 gives L+M = 53625.
    c = polya.counts(10, 2, 3, 4, 4, 1)
    assert c["L"] + c["M"] == 53625


def test_descending_lex_order():
    for l in range(1, 5):
        for d in range(0, 5):
            W = polya.monomials(l, d)
            for g, e in zip(W, W[1:]):
                diff = [a - b for a, b in zip(g, e)]
                first = next(x for x in diff if x != 0)
                assert first > 0
            assert W[0] == tuple([d] + [0] * (l - 1))


def test_printed_lex_formula_is_reversed():
    # eq. lex as printed enumerates ascending order; the adopted index is
    # f(l,d) + 1 minus it, which must be the position in W_d.
    for l in range(1, 5):
        for d in range(0, 5):
            W = polya.monomials(l, d)
            printed = [polya.lex_index_printed(g) for g in W]
            assert sorted(printed) == list(range(1, len(W) + 1))
            assert [polya.lex_index(g) for g in W] == list(range(1, len(W) + 1))
    # W_1 for l=2: (1,0) precedes (0,1) in the text; the printed formula gives 2, 1.
    assert polya.lex_index_printed((1, 0)) == 2 and polya.lex_index_printed((0, 1)) == 1


def test_beta_worked_example():
    rows = read_golden("beta_example.txt")
    l, dp, d1 = map(int, rows[0])
    want = [[int(x) for x in r] for r in rows[1:]]
    assert polya.beta_recursion(l, dp, d1) == want


def test_H_worked_example():
    rows = read_golden("H_example.txt")
    l, dp, da, d2 = map(int, rows[0])
    want, cur = [], None
    for r in rows[1:]:
        if r[0] == "h":
            cur = []
            want.append(cur)
        else:
            cur.append([int(x) for x in r])
    assert polya.coef_recursion(l, dp, da, d2) == want
    # and through H itself with distinct random A1, A2
    A = np.random.default_rng(0).standard_normal((2, 3, 3))
    H = polya.H_from_coef(want, A)
    assert np.array_equal(H[1, 0], A[0] + A[1])       # H_{1,2} = A1 + A2
    assert np.array_equal(H[3, 0], np.zeros((3, 3)))  # H_{1,4} = 0
    assert np.array_equal(H[3, 1], A[1])              # H_{2,4} = A2


def test_homogenize_worked_example():
    rng = np.random.default_rng(1)
    C, D, E, F = (rng.standard_normal((2, 2)) for _ in range(4))
    terms = {(2, 0, 0): C, (0, 1, 0): D, (0, 0, 1): E, (0, 0, 0): F}
    B = polya.homogenize(terms, 3)
    rows = read_golden("homogenize_example.txt")
    assert [tuple(map(int, r[:3])) for r in rows] == polya.monomials(3, 2)
    for r in rows:
        g = tuple(map(int, r[:3]))
        w = list(map(int, r[3:]))
        assert np.allclose(B[g], w[0] * C + w[1] * D + w[2] * E + w[3] * F, rtol=0, atol=1e-15)


@pytest.mark.parametrize("l,dp,d1", GRID)
def test_beta_three_ways(l, dp, d1):
    r = polya.beta_recursion(l, dp, d1)
    assert r == polya.beta_closed(l, dp, d1)
    assert r == polya.beta_bruteforce(l, dp, d1)
    for row in r:                                    # sum over g of beta = l^d1
        assert sum(row) == l ** d1


@pytest.mark.parametrize("l,dp,d2", GRID)
@pytest.mark.parametrize("da", [1, 2])
def test_coef_three_ways(l, dp, d2, da):
    r = polya.coef_recursion(l, dp, da, d2)
    assert r == polya.coef_closed(l, dp, da, d2)
    assert r == polya.coef_bruteforce(l, dp, da, d2)
    Na = polya.f(l, da)
    for rows in r:
        for lam in range(Na):
            assert sum(rows[g][lam] for g in range(len(rows))) == l ** d2


def _poly_eval(coeffs, mons, alpha):
    return sum(c * np.prod(alpha ** np.array(g)) for c, g in zip(coeffs, mons))


@pytest.mark.parametrize("l,dp,d", [(2, 1, 1), (3, 1, 2), (3, 2, 2), (4, 2, 1), (2, 3, 3)])
def test_polynomial_identities(l, dp, d):
    """(sum a)^d1 P(a) = sum_g (sum_h beta_{h,g} P_h) a^g and
    (sum a)^d2 (A^T P + P A)(a) = sum_g sum_h (H^T P_h + P_h H) a^g
    at random points, with A(a) = sum_i A_i a_i and random symmetric P_h."""
    rng = np.random.default_rng(7)
    n = 3
    A = rng.standard_normal((l, n, n))
    sdp = make_sdp(A, n, l, dp, d)
    Wp, WL, WM = polya.monomials(l, dp), polya.monomials(l, dp + d), polya.monomials(l, dp + 1 + d)
    Ps = [(lambda S: S + S.T)(rng.standard_normal((n, n))) for _ in Wp]
    for _ in range(5):
        a = rng.random(l)
        Pa = sum(P * np.prod(a ** np.array(h)) for P, h in zip(Ps, Wp))
        Aa = sum(A[i] * a[i] for i in range(l))
        lhs1 = a.sum() ** d * Pa
        rhs1 = sum(sum(sdp.beta[hi, j] * Ps[hi] for hi in range(len(Wp))) * np.prod(a ** np.array(g))
                   for j, g in enumerate(WL))
        assert np.allclose(lhs1, rhs1, rtol=1e-12, atol=1e-12)
        lhs2 = a.sum() ** d * (Aa.T @ Pa + Pa @ Aa)
        rhs2 = sum(sum(sdp.H[m, hi].T @ Ps[hi] + Ps[hi] @ sdp.H[m, hi] for hi in range(len(Wp)))
                   * np.prod(a ** np.array(g)) for m, g in enumerate(WM))
        assert np.allclose(lhs2, rhs2, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("l,dp,d", [(1, 1, 1), (2, 2, 3), (3, 1, 1), (4, 2, 2), (4, 1, 3)])
def test_block_scale_closed_form(l, dp, d):
    """eq. Cj: sum_h beta_{h,j} dp!/h! equals (dp+d1)!/g_j! (the coefficient of
    a^g in (sum a)^{dp+d1})."""
    sdp = make_sdp(np.zeros((l, 1, 1)), 1, l, dp, d)
    WL = polya.monomials(l, dp + d)
    for j, g in enumerate(WL):
        assert sdp.scale[j] == factorial(dp + d) / np.prod([factorial(x) for x in g])
    assert np.sum(sdp.scale[:sdp.L]) == l ** (dp + d)
    assert np.sum(sdp.scale[sdp.L:]) == l ** (dp + 1 + d)


def test_multinomial_and_overflow_bound():
    assert polya.multinomial(4, (2, 1, 1)) == 12
    # the largest Polya multinomial stays below 2^63 up to degree 20
    assert factorial(20) < 2 ** 63 < factorial(21)

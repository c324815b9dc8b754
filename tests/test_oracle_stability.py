"""Pins of the oracle's robust-stability driver (oracle/stability.py):

* the homogeneous representation (Section II) against the paper's worked
  example, and B(alpha) = A(G alpha) on the simplex as a polynomial identity;
* the translated-simplex maps of Section V (Examples 1 and 2): the images of
  the simplex's vertices are the corners of the printed regions;
* Example 2's printed matrices: the brute-force spectral boundary over a
  simplex grid reproduces the paper's L_opt = -0.111;
* the bisection: every certified L is sound (at or above the spectral
  boundary, and its certificate checks out at grid points), degrees only make
  it less conservative, and splitting each bracket in more than two parts
  ends in the same bracket.
"""
import numpy as np
import pytest

from conftest import read_golden
from oracle import ipm, polya, sdp as S, stability as St


def _example2():
    rows = read_golden("example2_matrices.txt")
    return np.array([[float(v) for v in r] for r in rows]).reshape(6, 3, 3)


def test_homogenization_worked_example():
    rng = np.random.default_rng(0)
    C, D, E, F = rng.standard_normal((4, 2, 2))
    B = St.poly_on_simplex([(2, 0, 0), (0, 1, 0), (0, 0, 1), (0, 0, 0)], np.stack([C, D, E, F]), None, 3, 2)
    rows = read_golden("homogenize_example.txt")
    W = polya.monomials(3, 2)
    for r in rows:
        g = tuple(int(v) for v in r[:3])
        w = [int(v) for v in r[3:]]
        want = w[0] * C + w[1] * D + w[2] * E + w[3] * F
        assert np.array_equal(B[W.index(g)], want)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_poly_on_simplex_identity(seed):
    """A random non-homogeneous A of degree <= 3 in 4 variables composed with
    a random linear map of the 3-simplex: B(alpha) = A(G alpha) on Delta_3."""
    rng = np.random.default_rng(seed)
    exps = [(0, 0, 0, 0), (1, 0, 0, 0), (0, 2, 0, 1), (1, 1, 1, 0), (0, 0, 0, 2), (3, 0, 0, 0)]
    mats = rng.standard_normal((len(exps), 3, 3))
    G = rng.standard_normal((4, 3))
    B = St.poly_on_simplex(exps, mats, G, 3, 3)
    for a in rng.dirichlet(np.ones(3), size=20):
        want = St.evaluate(exps, mats, G @ a)
        got = St.evaluate_homogeneous(B, 3, 3, a)
        assert np.abs(got - want).max() <= 1e-12 * (1 + np.abs(want).max())


def test_example2_map_corners():
    G0, G1 = St.example2_maps()
    for L in (-0.4, -0.111, 0.2):
        G = G0 + L * G1
        for i in range(3):
            x = G @ np.eye(3)[i]
            assert abs(x.sum() - (2 * L + 1)) <= 1e-15
            assert x[i] == 1.0 and all(abs(x[j] - L) <= 1e-16 for j in range(3) if j != i)


def test_example1_map_corners():
    """Example 1: g_i = 2 rho (alpha_i - 1/2) = rho (2 alpha_i - sum alpha) on
    the simplex; for l = 8 the region has coordinate sum -6 rho and
    -rho <= x_i <= rho."""
    l, rho = 8, 0.37
    G = rho * (2 * np.eye(l) - np.ones((l, l)))
    rng = np.random.default_rng(4)
    for a in rng.dirichlet(np.ones(l), size=10):
        x = G @ a
        assert abs(x.sum() + 6 * rho) <= 1e-14
        assert np.all(np.abs(x) <= rho + 1e-15)
        assert np.allclose(x, 2 * rho * (a - 0.5), atol=1e-15)


def test_example2_spectral_boundary_reproduces_printed_optimum():
    """The smallest L for which every grid point of S_L gives a Hurwitz A
    is the paper's L_opt = -0.111 (to the grid's resolution)."""
    G0, G1 = St.example2_maps()
    lb = St.spectral_boundary(St.EXAMPLE2_EXPS, _example2(), G0, G1, 3, 0.5, -0.5, 1e-4, 60)
    assert abs(lb - (-0.111)) <= 2e-3


def _certificate_holds(mats, L, r_y, dp, d, grid=20):
    """The FEASIBLE certificate's P(alpha) checked pointwise on a grid."""
    G0, G1 = St.example2_maps()
    Ap = St.poly_on_simplex(St.EXAMPLE2_EXPS, mats, G0 + L * G1, 3, 3)
    sdp = S.make_sdp(Ap, 3, 3, dp, d, da=3)
    P = sdp.P_of_y(r_y)
    Wp = polya.monomials(3, dp)
    for m in polya.monomials(3, grid):
        a = np.array(m, dtype=np.float64) / grid
        Pa = sum(P[i] * np.prod(a ** np.array(h)) for i, h in enumerate(Wp))
        Aa = St.evaluate_homogeneous(Ap, 3, 3, a)
        if np.linalg.eigvalsh(Pa)[0] <= 0 or np.linalg.eigvalsh(Aa.T @ Pa + Pa @ Aa)[-1] >= 0:
            return False
    return True


@pytest.mark.slow
def test_example2_bisection_sound_and_monotone():
    mats = _example2()
    G0, G1 = St.example2_maps()
    res = {}
    for dp, d in [(1, 1), (1, 2), (2, 2)]:
        r = St.bisect_simplex(St.EXAMPLE2_EXPS, mats, G0, G1, 3, dp, d, 0.5, -0.5, 2e-3)
        assert r.t_cert == r.t_cert and r.t_cert - r.t_other <= 2e-3
        res[(dp, d)] = r.t_cert
        # sound: never below the brute-force boundary
        assert r.t_cert >= -0.1117
        # the last certified trial's P checks out pointwise
        Ap = St.poly_on_simplex(St.EXAMPLE2_EXPS, mats, G0 + r.t_cert * G1, 3, 3)
        o = ipm.ipm_solve(S.make_sdp(Ap, 3, 3, dp, d, da=3))
        assert o.verdict == ipm.FEASIBLE
        assert _certificate_holds(mats, r.t_cert, o.y, dp, d)
    # higher degrees are never more conservative (up to the bracket width)
    assert res[(1, 2)] <= res[(1, 1)] + 2e-3
    assert res[(2, 2)] <= res[(1, 2)] + 2e-3


def test_multisection_same_bracket():
    """Three trials per round instead of one: the final brackets (width <=
    tol, both containing the SDP's own threshold) overlap."""
    mats = _example2()
    G0, G1 = St.example2_maps()
    r1 = St.bisect_simplex(St.EXAMPLE2_EXPS, mats, G0, G1, 3, 0, 1, 0.5, -0.5, 4e-3)
    r3 = St.bisect_simplex(St.EXAMPLE2_EXPS, mats, G0, G1, 3, 0, 1, 0.5, -0.5, 4e-3, width=3)
    assert abs(r1.t_cert - r3.t_cert) <= 4e-3
    assert min(r1.t_cert, r3.t_cert) >= max(r1.t_other, r3.t_other) - 1e-15
    # a round of three trials (one batch on the device) shrinks the bracket
    # four times: fewer rounds than plain bisection
    rounds1, rounds3 = len(r1.trials) - 1, (len(r3.trials) - 1) // 3
    assert (len(r3.trials) - 1) % 3 == 0 and rounds3 < rounds1

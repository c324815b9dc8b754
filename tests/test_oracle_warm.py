"""Warm-start projection and fallback of the oracle IPM (CPU).

The warm start is not part of the paper: these pins fix its definition
(closed forms of the projection) and its contract (the cold pipeline's
answer whenever the warm run is rejected; the same optimum when accepted).
"""
import numpy as np
import pytest

from oracle import ipm, sdp as S
from paper_1411_3769_amd import workloads as W


@pytest.fixture(scope="module")
def plain():
    sy = W.plain_system(2)
    return S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)


@pytest.mark.parametrize("center", [True, False])
def test_projection_closed_form(plain, center):
    rng = np.random.default_rng(0)
    y0 = 1e-3 * rng.standard_normal(plain.K)
    s = rng.uniform(-3, 1, plain.nb)
    X, y, Z = ipm.warm_start_point(plain, y0, s, margin=1e-4, center=center)
    Wb = plain.BT(y0) - plain.C_blocks()
    I = np.eye(plain.n)
    for j in range(plain.nb):
        lw = np.linalg.eigvalsh(Wb[j])[0]
        D = Z[j] - Wb[j]
        tau = D[0, 0]
        assert np.allclose(D, tau * I, atol=1e-15)                  # a multiple of I
        assert abs(np.linalg.eigvalsh(Z[j])[0] - max(lw, 1e-4 * plain.scale[j])) <= 1e-12
        assert abs(np.trace(X[j]) - plain.n * np.exp(s[j])) <= 1e-12 * np.trace(X[j])
        if center:                                                 # Z X = c I
            ZX = Z[j] @ X[j]
            c = plain.n * np.exp(s[j]) / np.trace(np.linalg.inv(Z[j]))
            assert np.allclose(ZX, c * I, atol=1e-10 * c)
        else:
            assert np.allclose(X[j], np.exp(s[j]) * I)
    assert np.array_equal(y, y0)


def test_interior_start_is_kept(plain):
    """A start already inside by more than the margin is not moved."""
    r = ipm.ipm_run(ipm.PaperOps(plain), ipm.Options(), max_iter=8)
    Wb = plain.BT(r.y) - plain.C_blocks()
    lam = min(np.linalg.eigvalsh(Wb[j])[0] for j in range(plain.nb))
    assert lam > 1e-6 * plain.scale.max()
    X, y, Z = ipm.warm_start_point(plain, r.y, None, margin=1e-6)
    assert np.array_equal(Z, Wb)


def test_warm_from_trajectory_reaches_same_optimum(plain):
    cold = ipm.ipm_solve(plain)
    assert cold.verdict == ipm.FEASIBLE
    k = 10
    mid = ipm.ipm_run(ipm.PaperOps(plain), ipm.Options(), max_iter=k)
    logx = np.log(np.trace(mid.X, axis1=1, axis2=2) / plain.n)
    w = ipm.ipm_solve(plain, warm=(mid.y, logx))
    assert w.warm_used and not w.warm_fallback
    assert w.verdict == ipm.FEASIBLE
    assert abs(w.psi - cold.psi) <= 1e-6 * abs(cold.psi)
    assert w.iterations < cold.iterations


def test_rejected_warm_start_falls_back_to_cold(plain):
    cold = ipm.ipm_solve(plain)
    rng = np.random.default_rng(1)
    w = ipm.ipm_solve(plain, warm=(rng.standard_normal(plain.K), None), warm_iter_cap=2)
    assert w.warm_fallback and not w.warm_used and w.warm_iterations == 2
    assert w.verdict == cold.verdict and w.psi == cold.psi and w.iterations == cold.iterations

"""GPU parity of the robust-stability driver (Section V, Examples 1 and 2)
against the oracle (marker: gpu):

* psdp_poly_on_simplex (homogeneous representation of A on a translated
  simplex, Section II) against the oracle's expansion;
* the set-up of systems of degree da = 2 and 3 (eq. H_init with |lambda| = da)
  bit for bit;
* psdp_bisect_simplex on Example 2's printed system: the same trial values
  and verdicts as the oracle's bisection, plain and with several trials per
  round, and a certified L that is sound (never below the brute-force
  spectral boundary of the printed L_opt = -0.111).
"""
import numpy as np
import pytest

from conftest import read_golden
from oracle import ipm, polya, sdp as S, stability as St

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _example2():
    rows = read_golden("example2_matrices.txt")
    return np.array([[float(v) for v in r] for r in rows]).reshape(6, 3, 3)


@pytest.mark.parametrize("L", [-0.3, -0.111, 0.05, 0.4])
def test_poly_on_simplex_example2(P, L):
    mats = _example2()
    G0, G1 = St.example2_maps()
    got = P.poly_on_simplex(St.EXAMPLE2_EXPS, mats, G0 + L * G1, 3, 3)
    want = St.poly_on_simplex(St.EXAMPLE2_EXPS, mats, G0 + L * G1, 3, 3)
    assert np.abs(got - want).max() <= 4e-16 * np.abs(want).max()


def test_poly_on_simplex_homogenization(P):
    """Section II's construction (identity map, a constant term)."""
    rng = np.random.default_rng(5)
    exps = [(2, 0, 0), (0, 1, 0), (0, 0, 1), (0, 0, 0)]
    mats = rng.standard_normal((4, 3, 3))
    assert np.array_equal(P.poly_on_simplex(exps, mats, None, 3, 2),
                          St.poly_on_simplex(exps, mats, None, 3, 2))


@pytest.mark.parametrize("n,l,dp,d,da", [(3, 3, 1, 1, 3), (3, 3, 2, 2, 3), (4, 3, 1, 2, 2), (5, 4, 1, 1, 2)])
def test_setup_higher_degree_bit_exact(P, n, l, dp, d, da):
    rng = np.random.default_rng(n * 10 + da)
    A = rng.standard_normal((polya.f(l, da), n, n))
    g = P.polya_setup(A, n, l, dp, d, da=da)
    o = S.make_sdp(A, n, l, dp, d, da=da)
    got = g.get_polya()
    assert (g.L0, g.L, g.M, g.K, g.Na) == (o.L0, o.L, o.M, o.K, polya.f(l, da))
    assert np.array_equal(got["beta"], np.array(polya.beta_closed(l, dp, d), dtype=np.int64))
    assert np.array_equal(got["coef"], np.array(polya.coef_closed(l, dp, da, d), dtype=np.int64))
    assert np.array_equal(got["H"].view(np.uint64), o.H.view(np.uint64))
    assert np.array_equal(got["scale"], o.scale)
    assert np.array_equal(got["cdiag"], o.cdiag)


@pytest.mark.parametrize("dp,d,width", [(1, 1, 1), (1, 2, 1), (1, 2, 4), (2, 2, 3)])
def test_bisection_example2(P, dp, d, width):
    print(f"bisection dp={dp} d={d} width={width}", flush=True)
    mats = _example2()
    G0, G1 = St.example2_maps()
    tol = 2e-3
    r = P.bisect_simplex(St.EXAMPLE2_EXPS, mats, G0, G1, 3, dp, d, 0.5, -0.5, tol, width=width)
    o = St.bisect_simplex(St.EXAMPLE2_EXPS, mats, G0, G1, 3, dp, d, 0.5, -0.5, tol, width=width)
    # the same trials: identical points as long as every verdict agrees (the
    # iteration counts of trials near the threshold, which stall and go to
    # phase-I, depend on the trajectory and are not compared)
    assert len(r.trials) == len(o.trials)
    for (t, v, it, _), (to, vo, ito) in zip(r.trials, o.trials):
        assert t == to and v == vo, (t, v, to, vo)
    assert r.t_cert == o.t_cert and r.t_other == o.t_other
    assert abs(r.t_cert - r.t_other) <= tol
    assert r.t_cert >= -0.1117     # sound: the printed optimum is -0.111

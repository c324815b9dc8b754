"""GPU parity of the discrete-time form (x+ = A(alpha) x as an instance of the
generalized LMI of Section III-C; blocks of order 2n) against the oracle's
DiscretePolyaSDP (marker: gpu):

* set-up bit for bit (beta, the H weights and H, scales, C);
* the Newton step at fixed positive definite iterates: Z^-1, B^T(y), B(X),
  the Schur complement (by the oracle's definition), its factor and a solve,
  on blocks of order 2n <= 16 (the small-block kernels) and > 16 (the
  general kernels and the grouped assembly's copy terms);
* end to end: the scalar closed form max(delta, eps/(1-|a|)), a contractive
  polytope certified with the oracle's objective and margin, an unstable
  vertex refuted as by the oracle, the Hurwitz / Schur separation, the FP32
  assembly form, and a batch mixing both forms in one solve.
"""
import numpy as np
import pytest

from oracle import discrete as D, ipm, polya, sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _perm(g, n, L0):
    pairs = g.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


@pytest.mark.parametrize("n,l,dp,d", [(1, 3, 0, 1), (3, 3, 1, 1), (5, 2, 2, 1), (9, 2, 1, 1)])
def test_setup_bit_exact(P, n, l, dp, d):
    A = np.random.default_rng(n * 10 + l).standard_normal((l, n, n))
    g = P.polya_setup(A, n, l, dp, d, form="discrete")
    o = D.make_discrete_sdp(A, n, l, dp, d)
    assert g.form == "discrete" and g.bo == 2 * n and (g.K, g.L0, g.L, g.M) == (o.K, o.L0, o.L, o.M)
    got = g.get_polya()
    assert np.array_equal(got["H"].view(np.uint64), o.H.view(np.uint64))
    assert np.array_equal(got["scale"], o.scale)
    assert np.array_equal(got["cdiag"], o.cdiag)


NEWTON = [(1, 3, 1, 1, 0), (3, 3, 1, 1, 1), (4, 2, 1, 2, 2), (8, 2, 1, 1, 3), (9, 2, 1, 1, 4),
          (12, 3, 1, 1, 5)]


@pytest.mark.parametrize("n,l,dp,d,seed", NEWTON)
def test_newton_step_parity(P, n, l, dp, d, seed):
    print(f"discrete newton n={n} l={l} dp={dp} d={d}", flush=True)
    rng = np.random.default_rng(seed)
    A = 0.4 * rng.standard_normal((l, n, n))
    g = P.polya_setup(A, n, l, dp, d, form="discrete")
    o = D.make_discrete_sdp(A, n, l, dp, d)
    X = W.random_spd_blocks(seed + 1, o.nb, 2 * n)
    Z = W.random_spd_blocks(seed + 2, o.nb, 2 * n)
    y_or = rng.standard_normal(o.K)
    perm = _perm(g, n, o.L0)
    out = P.eval_newton(g, X, Z, y_or[perm])
    Zi = np.linalg.inv(Z)
    assert np.abs(out["Zi"] - Zi).max() <= 1e-12 * np.abs(Zi).max()
    BT = o.BT(y_or)
    assert np.abs(out["BTy"] - BT).max() <= 1e-12 * np.abs(BT).max()
    BX = o.B(X)[perm]
    assert np.abs(out["BX"] - BX).max() <= 1e-12 * np.abs(BX).max()
    Lam = S.schur_definition(o, X, Zi)[np.ix_(perm, perm)]
    sc = np.abs(Lam).max()
    assert np.abs(out["Lam"] - Lam).max() <= 1e-12 * sc
    Lf = out["LamL"]
    assert np.abs(Lf @ Lf.T - Lam).max() <= 1e-11 * sc
    x = np.linalg.solve(Lam, y_or[perm])
    assert np.abs(out["sol"] - x).max() <= 1e-9 * np.abs(x).max()


def _match(r, o, tol=1e-6):
    assert r.verdict == o.verdict, (r.verdict_name, o.verdict)
    if o.verdict == ipm.FEASIBLE and not o.phase1_used:
        for k in ("psi", "phi", "margin"):
            assert abs(getattr(r, k) - getattr(o, k)) <= tol * abs(getattr(o, k)), (k, getattr(r, k), getattr(o, k))


@pytest.mark.parametrize("a", [0.5, -0.7, 0.9])
def test_scalar_closed_form(P, a):
    g = P.polya_setup(np.full((3, 1, 1), a), 1, 3, 0, 1, form="discrete")
    r = P.ipm_solve(g)
    assert r.verdict_name == "FEASIBLE"
    want = max(1e-3, 1e-3 / (1 - abs(a)))
    assert abs(r.psi - want) <= 1e-6 * want


def _contractive(rng, l, n, rho):
    out = []
    for _ in range(l):
        Q = rng.standard_normal((n, n))
        out.append(rho * Q / np.linalg.norm(Q, 2))
    return np.stack(out)


@pytest.mark.parametrize("asm_path", [0, 1])
@pytest.mark.parametrize("seed,n,dp,d", [(0, 3, 1, 1), (1, 6, 1, 1), (2, 10, 1, 1)])
def test_contractive_polytope(P, seed, n, dp, d, asm_path):
    """Both assembly kernels (grouped tiles; whole pairs, n^2 <= 128) read
    the copy terms."""
    rng = np.random.default_rng(seed)
    A = _contractive(rng, 3, n, 0.9)
    print(f"discrete contractive n={n} asm_path={asm_path}", flush=True)
    o = ipm.ipm_solve(D.make_discrete_sdp(A, n, 3, dp, d))
    r = P.ipm_solve(P.polya_setup(A, n, 3, dp, d, form="discrete"), asm_path=asm_path)
    _match(r, o)
    assert r.verdict_name == "FEASIBLE" and r.asm_path == asm_path


def test_unstable_vertex(P):
    rng = np.random.default_rng(3)
    A = _contractive(rng, 3, 2, 0.5)
    A[1] = np.array([[1.1, 0.3], [0.0, 0.2]])
    o = ipm.ipm_solve(D.make_discrete_sdp(A, 2, 3, 1, 2))
    r = P.ipm_solve(P.polya_setup(A, 2, 3, 1, 2, form="discrete"))
    assert r.verdict == o.verdict and r.verdict_name != "FEASIBLE"


def test_forms_separate(P):
    hur = np.stack([-2.0 * np.eye(2), -2.0 * np.eye(2) + [[0, 0.1], [0, 0]]])
    sch = np.stack([0.5 * np.eye(2), 0.5 * np.eye(2) + [[0, 0.1], [0, 0]]])
    v = lambda A, f: P.ipm_solve(P.polya_setup(A, 2, 2, 0, 1, form=f)).verdict_name
    assert v(hur, "continuous") == "FEASIBLE" and v(hur, "discrete") != "FEASIBLE"
    assert v(sch, "continuous") != "FEASIBLE" and v(sch, "discrete") == "FEASIBLE"


def test_fp32_assembly_form(P):
    rng = np.random.default_rng(4)
    A = _contractive(rng, 3, 10, 0.85)
    o = ipm.ipm_solve(D.make_discrete_sdp(A, 10, 3, 1, 1))
    r = P.ipm_solve(P.polya_setup(A, 10, 3, 1, 1, form="discrete"), precision="fp32")
    _match(r, o)
    assert r.iters_lowprec >= 1


def test_mixed_forms_in_one_batch(P):
    """Continuous and discrete systems (blocks of order n and 2n) solved
    together; each matches its own oracle."""
    rng = np.random.default_rng(6)
    cases = []
    for i in range(6):
        n = 2 + i
        if i % 2 == 0:
            A = _contractive(rng, 3, n, 0.8)
            cases.append(("discrete", A, n, D.make_discrete_sdp(A, n, 3, 1, 1)))
        else:
            A = rng.standard_normal((3, n, n)) * 0.3 - 1.5 * np.eye(n)
            cases.append(("continuous", A, n, S.make_sdp(A, n, 3, 1, 1)))
    gs = [P.polya_setup(A, n, 3, 1, 1, form=f) for f, A, n, _ in cases]
    rs = P.ipm_solve_batched(gs)
    for (f, A, n, o), r in zip(cases, rs):
        _match(r, ipm.ipm_solve(o))

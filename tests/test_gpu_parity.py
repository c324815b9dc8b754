"""GPU parity of the HIP path against the FP64 oracle (marker: gpu).

Bit-exact: beta, the integer H weights, H itself, the block scales and C.
FP64 hot-path steps at fixed positive definite iterates: Z^{-1}, B^T(y),
B(X), the Schur complement, its Cholesky factor and a solve (relative 1e-12;
the factor by the right-looking tiled form, with and without sub-panels, and
by the left-looking one), and
the step ladder (identical rung).  End to end: same verdict, objective
and certificate margin within 1e-6 relative.
"""
import json
import os

import numpy as np
import pytest

from conftest import GOLDEN
from oracle import ipm, polya, sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _flush(msg):
    print(msg, flush=True)


def _perm(sdp_gpu, n, L0):
    """Library dual index -> oracle dual index."""
    pairs = sdp_gpu.basis()
    opos = {pq: b for b, pq in enumerate(S.basis_pairs(n))}
    Nt = n * (n + 1) // 2
    bmap = np.array([opos[(int(p), int(q))] for p, q in pairs])
    return np.concatenate([h * Nt + bmap for h in range(L0)])


SETUP_CASES = [(4, 3, 1, 1), (10, 4, 2, 2), (3, 2, 3, 2), (1, 3, 2, 2), (9, 2, 1, 3), (17, 3, 1, 1),
               (5, 1, 2, 4), (100, 4, 1, 3)]


@pytest.mark.parametrize("n,l,dp,d", SETUP_CASES)
def test_polya_setup_bit_exact(P, n, l, dp, d):
    _flush(f"setup n={n} l={l} dp={dp} d={d}")
    A = np.random.default_rng(n * 100 + l).standard_normal((l, n, n))
    g = P.polya_setup(A, n, l, dp, d)
    o = S.make_sdp(A, n, l, dp, d)
    got = g.get_polya()
    assert (g.L0, g.L, g.M, g.K) == (o.L0, o.L, o.M, o.K)
    assert np.array_equal(got["beta"], np.array(polya.beta_closed(l, dp, d), dtype=np.int64))
    assert np.array_equal(got["coef"], np.array(polya.coef_closed(l, dp, 1, d), dtype=np.int64))
    assert np.array_equal(got["H"].view(np.uint64), o.H.view(np.uint64))
    assert np.array_equal(got["scale"], o.scale)
    assert np.array_equal(got["cdiag"], o.cdiag)


NEWTON_CASES = [(4, 3, 1, 1, 0), (10, 4, 2, 2, 1), (3, 2, 2, 1, 2), (9, 2, 1, 2, 3), (13, 2, 1, 1, 4),
                (1, 3, 1, 1, 5), (20, 3, 1, 1, 6)]
# Schur matrices of 22, 33 and 56 tiles of 64: the factorisation's depth-512
# wide updates run, the first two with a last super-panel that absorbs a
# short trailing run; the solves go by groups of 16 tiles, the last one
# partial in each (6, 1 and 8 tiles)
NEWTON_BIG = [(16, 4, 2, 1, 7), (32, 4, 1, 2, 8), (48, 3, 1, 1, 9)]


# factorisations: default right-looking (width 8), left-looking, panel
# solves folded into the updates, look-ahead steps, and widths 16 / 8 split in
# sub-panels of 4 (sub-panel updates of depth 256)
@pytest.mark.parametrize("chol", [(0, 0), (-1, 0), (-2, 0), (-3, 0), (16, 4), (8, 4)])
@pytest.mark.parametrize("n,l,dp,d,seed", NEWTON_CASES + NEWTON_BIG)
def test_newton_step_parity(P, n, l, dp, d, seed, chol):
    _flush(f"newton n={n} l={l} dp={dp} d={d} seed={seed} chol_panels={chol}")
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((l, n, n)) - 1.5 * np.eye(n)
    g = P.polya_setup(A, n, l, dp, d)
    o = S.make_sdp(A, n, l, dp, d)
    X = W.random_spd_blocks(seed + 1, o.nb, n)
    Z = W.random_spd_blocks(seed + 2, o.nb, n)
    y_or = rng.standard_normal(o.K)
    perm = _perm(g, n, o.L0)
    y_lib = y_or[perm]
    out = P.eval_newton(g, X, Z, y_lib, chol_panels=chol[0], chol_subpanels=chol[1])
    Zi = np.linalg.inv(Z)
    assert np.abs(out["Zi"] - Zi).max() <= 1e-12 * np.abs(Zi).max()
    BT = o.BT(y_or)
    assert np.abs(out["BTy"] - BT).max() <= 1e-12 * np.abs(BT).max()
    BX = o.B(X)[perm]
    assert np.abs(out["BX"] - BX).max() <= 1e-12 * np.abs(BX).max()
    if o.K <= 700:
        # the definition of every column, B(Z^-1 B^T(e_l) X)
        Lam = S.schur_definition(o, X, Zi)[np.ix_(perm, perm)]
    else:
        # the expanded form everywhere, the definition on columns spread over
        # every tile (first and last column of each, in the library's order)
        Lam = S.schur_expanded(o, X, Zi)[np.ix_(perm, perm)]
        cols = sorted({c for t in range(0, o.K, 64) for c in (t, min(t + 63, o.K - 1))})
        Ld = S.schur_definition_columns(o, X, Zi, [int(perm[c]) for c in cols])[perm]
        assert np.abs(out["Lam"][:, cols] - Ld).max() <= 1e-12 * np.abs(Ld).max()
    sc = np.abs(Lam).max()
    assert np.abs(out["Lam"] - Lam).max() <= 1e-12 * sc
    Lf = out["LamL"]
    assert np.abs(Lf @ Lf.T - Lam).max() <= 1e-11 * sc
    x = np.linalg.solve(Lam, y_lib)
    assert np.abs(out["sol"] - x).max() <= 1e-9 * np.abs(x).max()


@pytest.mark.parametrize("n", [65, 100, 128])
def test_block_inverse_tile_orders(P, n):
    """Z^{-1} and B^T(y) of blocks of order 64 < n <= 128 (the tile
    factorisation of Z padded to 128; B^T's tiled block products) against
    numpy's inverse and the oracle's operator."""
    _flush(f"block inverse n={n}")
    rng = np.random.default_rng(n)
    A = rng.standard_normal((2, n, n)) - 1.5 * np.eye(n)
    g = P.polya_setup(A, n, 2, 1, 1)
    o = S.make_sdp(A, n, 2, 1, 1)
    X = W.random_spd_blocks(n + 1, o.nb, n)
    Z = W.random_spd_blocks(n + 2, o.nb, n)
    y_or = rng.standard_normal(o.K)
    out = P.eval_newton(g, X, Z, y_or[_perm(g, n, o.L0)], schur=False)
    Zi = np.linalg.inv(Z)
    assert np.abs(out["Zi"] - Zi).max() <= 1e-11 * np.abs(Zi).max()
    assert np.array_equal(out["Zi"], np.transpose(out["Zi"], (0, 2, 1)))
    BT = o.BT(y_or)
    assert np.abs(out["BTy"] - BT).max() <= 1e-12 * np.abs(BT).max()


@pytest.mark.parametrize("n", [65, 128])
def test_certificate_tile_orders(P, n):
    """The certificate of blocks of order 64 < n <= 128 (each bisection test
    the tile Cholesky of the block padded with the identity to 128): every
    block of B^T(y) positive definite and the margin equal to
    min_j lambda_min(B^T(y)_j) / s_j through the oracle's operators."""
    _flush(f"certificate n={n}")
    sy = W.paper_shape_system(n, 2, seed=n)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g)
    assert r.verdict_name == "FEASIBLE" and not r.phase1_used, (r.verdict_name, r.reason_name)
    o = S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d)
    y = np.empty_like(r.y)
    y[_perm(g, n, o.L0)] = r.y
    Q = o.BT(y)
    lam = np.array([np.linalg.eigvalsh(Q[j])[0] for j in range(o.nb)])
    assert lam.min() > 0
    assert abs(r.margin - float(np.min(lam / o.scale))) <= 1e-6 * abs(r.margin)


@pytest.mark.parametrize("n,l,dp,d,seed", NEWTON_CASES)
def test_lookahead_equals_right_looking(P, n, l, dp, d, seed):
    """The look-ahead steps compute every value as the right-looking steps of
    one super-panel do (the diagonal factorisation repeated in each workgroup
    of the next column gives the same bits), so factor and solution agree bit
    for bit."""
    _flush(f"look-ahead n={n} l={l} dp={dp} d={d} seed={seed}")
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((l, n, n)) - 1.5 * np.eye(n)
    g = P.polya_setup(A, n, l, dp, d)
    o = S.make_sdp(A, n, l, dp, d)
    X = W.random_spd_blocks(seed + 1, o.nb, n)
    Z = W.random_spd_blocks(seed + 2, o.nb, n)
    y = rng.standard_normal(o.K)
    a = P.eval_newton(g, X, Z, y, chol_panels=32)
    b = P.eval_newton(g, X, Z, y, chol_panels=-3)
    assert np.array_equal(a["LamL"], b["LamL"])
    assert np.array_equal(a["sol"], b["sol"])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ladder_parity(P, seed):
    _flush(f"ladder seed={seed}")
    rng = np.random.default_rng(seed)
    sy = W.plain_system(seed)
    g = P.polya_setup(sy.A, 4, 3, 1, 1)
    o = S.make_sdp(sy.A, 4, 3, 1, 1)
    V = W.random_spd_blocks(seed, o.nb, 4)
    dV = rng.standard_normal((o.nb, 4, 4)) * (seed + 1)
    dV = dV + dV.transpose(0, 2, 1)
    step, k = P.eval_ladder(g, V, dV)
    want = ipm.ladder(V, dV, ipm.Options())
    assert step == want
    assert k >= 0


def _golden():
    with open(os.path.join(GOLDEN, "oracle_results.json")) as fh:
        return json.load(fh)


def _check_against(rec, r):
    assert r.verdict_name == rec["verdict"], (rec, r.verdict_name, r.reason_name)
    if rec["verdict"] == "FEASIBLE" and not rec["phase1_used"]:
        assert abs(r.psi - rec["psi"]) <= 1e-6 * abs(rec["psi"])
        assert abs(r.phi - rec["phi"]) <= 1e-6 * abs(rec["phi"])
        assert abs(r.margin - rec["margin"]) <= 1e-6 * abs(rec["margin"])
        assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
        # the trajectories differ by rounding only: a ladder rung on the
        # Cholesky boundary can shift the count by one
        assert abs(r.iterations - rec["iterations"]) <= 1, (r.iterations, rec["iterations"])


def test_plain_seeds_end_to_end(P):
    recs = [r for r in _golden() if r["tag"] == "plain"]
    for rec in recs:
        sy = W.plain_system(rec["seed"])
        _flush(f"plain seed={rec['seed']}")
        g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
        r = P.ipm_solve(g)
        _check_against(rec, r)


def test_twins_end_to_end(P):
    recs = [r for r in _golden() if r["tag"] == "plain-twin"]
    for rec in recs[:8]:
        sy = W.plain_system(rec["seed"], twin=True)
        _flush(f"twin seed={rec['seed']}")
        g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
        r = P.ipm_solve(g)
        _check_against(rec, r)
        if rec["phase1_used"]:
            assert abs(r.t_star - rec["t_star"]) <= 1e-6 * max(1e-3, abs(rec["t_star"]))


def test_n10_batch_of_64(P):
    recs = {r["seed"]: r for r in _golden() if r["tag"] == "n10"}
    sys_ = [W.c1_system(s) for s in range(64)]
    _flush("n10 batch of 64")
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    rs = P.ipm_solve_batched(gs)
    for s, r in enumerate(rs):
        _check_against(recs[s], r)


def test_batch_equals_single(P):
    sys_ = [W.c1_system(s) for s in range(3)] + [W.plain_system(5)]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    _flush("batch vs single")
    rb = P.ipm_solve_batched(gs)
    for g, r in zip(gs, rb):
        r1 = P.ipm_solve(g)
        assert r1.verdict == r.verdict and r1.iterations == r.iterations
        assert np.array_equal(r1.y, r.y)


def test_certificate_sound_on_simplex(P):
    sy = W.plain_system(0)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g)
    assert r.verdict == P.FEASIBLE
    Wp = polya.monomials(sy.l, sy.dp)
    rng = np.random.default_rng(3)
    for a in rng.dirichlet(np.ones(sy.l), size=3000):
        Pa = sum(r.P[i] * np.prod(a ** np.array(h)) for i, h in enumerate(Wp))
        Aa = np.tensordot(a, sy.A, axes=1)
        assert np.linalg.eigvalsh(Pa)[0] > 0
        assert np.linalg.eigvalsh(Aa.T @ Pa + Pa @ Aa)[-1] < 0


@pytest.mark.parametrize("a", [0.2, 2.0])
def test_scaled_identity_closed_form(P, a):
    n, l, dp, d = 5, 3, 1, 1
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    g = P.polya_setup(A, n, l, dp, d)
    r = P.ipm_solve(g)
    want = l ** dp * n * max(1e-3, 1e-3 / (2 * a))
    assert r.verdict == P.FEASIBLE
    assert abs(r.psi - want) <= 1e-6 * want


def test_scalar_case(P):
    g = P.polya_setup(-np.array([[[0.5]], [[1.0]], [[2.0]]]), 1, 3, 1, 1)
    assert P.ipm_solve(g).verdict == P.FEASIBLE

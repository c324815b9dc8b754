"""GPU parity of the solver's less-travelled branches against the FP64 oracle
(marker: gpu).  Each case runs the same option on both sides:

* the Schur factorisation's diagonal shift with refinement against the
  unshifted matrix-free product (Alg. 2, root step 1, with the failure policy
  of the design notes), forced on every step, and the shift cap;
* the phase-I margin SDP on feasible systems (t* > 0 and the certificate it
  rescales onto the paper's constraint), on the infeasible twin, and for a
  scalar system with one unstable vertex;
* the paper-literal set-up (derivative blocks C_j = 0, eq. Cj as printed)
  with the paper's absolute gap test (Section IV-A);
* Mehrotra's centring parameter.

End points are compared (verdict, objective, margin, normalised margin t*);
the trajectory itself may differ where a ladder rung sits on the Cholesky
boundary, so iteration counts are allowed to differ by one.
"""
import numpy as np
import pytest

from oracle import ipm, sdp as S
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _flush(msg):
    print(msg, flush=True)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def _same_end_point(r, o, its=1, margin="margin"):
    assert r.verdict == o.verdict, (r.verdict_name, r.reason_name, o.verdict, o.reason)
    if o.verdict == ipm.FEASIBLE:
        assert _rel(r.psi, o.psi) <= 1e-6, (r.psi, o.psi)
        assert _rel(getattr(r, margin), getattr(o, margin)) <= 1e-6, (getattr(r, margin), getattr(o, margin))
    assert abs(r.iterations - o.iterations) <= its, (r.iterations, o.iterations)
    assert r.phase1_used == o.phase1_used
    if o.phase1_used:
        # a phase-I run that does not converge ends wherever its trajectory
        # fails; only a converged run's length is comparable
        assert (r.phase1_reason == 0) == (o.phase1_reason == ipm.CONVERGED)
        if o.phase1_reason == ipm.CONVERGED:
            assert abs(r.phase1_iterations - o.phase1_iterations) <= its
        assert abs(r.t_star - o.t_star) <= 1e-6 * max(1e-3, abs(o.t_star)), (r.t_star, o.t_star)


@pytest.mark.parametrize("force", [1e-12, 1e-8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forced_shift(P, force, seed):
    _flush(f"forced shift {force:g} seed={seed}")
    sy = W.plain_system(seed)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, chol_shift_force=force)
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(shift_force=force))
    _same_end_point(r, o)
    assert r.verdict == P.FEASIBLE and r.reason_name == "converged"
    # every Newton step factored with the shift, each refined
    assert r.chol_shifts == r.iterations and o.chol_shifts == o.iterations
    assert r.ir_steps >= 1
    assert r.gap_rel <= 1e-8 and r.pinf <= 1e-8 and r.dinf <= 1e-8
    # the unshifted run: no shift, no refinement
    r0 = P.ipm_solve(g)
    assert r0.chol_shifts == 0 and r0.ir_steps == 0
    assert _rel(r.psi, r0.psi) <= 2e-8


def test_forced_shift_batch_mixes_with_unshifted(P):
    """A batch in which the shift is forced equals the single solves under the
    same option (the shifted kernels and refinement are per system)."""
    sys_ = [W.plain_system(3), W.c1_system(0), W.plain_system(4, twin=True)]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    _flush("forced shift batch")
    rb = P.ipm_solve_batched(gs, chol_shift_force=1e-10)
    for sy, g, r in zip(sys_, gs, rb):
        r1 = P.ipm_solve(g, chol_shift_force=1e-10)
        assert r1.verdict == r.verdict and r1.iterations == r.iterations
        assert r1.chol_shifts == r.chol_shifts
        assert np.array_equal(r1.y, r.y)
        o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(shift_force=1e-10))
        _same_end_point(r, o)


def test_shift_beyond_cap(P):
    """A forced shift above the cap leaves no factorisation to try: both runs
    end at their first Newton step with a Cholesky failure, and phase-I
    (which fails the same way) cannot decide."""
    sy = W.plain_system(0)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, chol_shift_force=1e-8, chol_shift_max=1e-9)
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d),
                      ipm.Options(shift_force=1e-8, shift_max=1e-9))
    assert o.reason == ipm.CHOL_FAIL and o.iterations == 0 and o.verdict == ipm.UNKNOWN
    assert r.reason_name == "chol_fail" and r.iterations == 0 and r.verdict == P.UNKNOWN
    assert r.phase1_used and r.phase1_iterations == 0 and r.chol_shifts == 0


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_phase1_only_feasible(P, seed):
    """Plain seeds decided by the phase-I margin SDP: t* > 0, the rescaled
    certificate passes with margin delta (some block attains t*), and its
    objective matches the oracle's rescaled certificate."""
    _flush(f"phase1_only seed={seed}")
    sy = W.plain_system(seed)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, verdict_mode="phase1_only")
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(verdict_mode="phase1_only"))
    assert o.verdict == ipm.FEASIBLE and o.t_star > 0
    assert r.iterations == 0 and o.iterations == 0
    _same_end_point(r, o)
    assert _rel(r.margin, 1e-3) <= 1e-6


@pytest.mark.parametrize("a", [0.2, 2.0])
def test_phase1_only_closed_form(P, a):
    """A_i = -aI: t* = delta / v* with v* = l^dp n delta max(1, 1/(2a)), and
    the rescaled certificate has objective v* (homogeneity of the optimum)."""
    n, l, dp, d = 3, 3, 1, 1
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    g = P.polya_setup(A, n, l, dp, d)
    r = P.ipm_solve(g, verdict_mode="phase1_only")
    v_star = l ** dp * n * 1e-3 * max(1.0, 1.0 / (2 * a))
    assert r.verdict == P.FEASIBLE and r.phase1_used
    assert _rel(r.t_star, 1e-3 / v_star) <= 1e-6
    assert _rel(r.psi, v_star) <= 1e-6


@pytest.mark.parametrize("seed", [0, 1])
def test_phase1_only_twin(P, seed):
    sy = W.plain_system(seed, twin=True)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, verdict_mode="phase1_only")
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(verdict_mode="phase1_only"))
    assert o.verdict == ipm.INFEASIBLE
    _same_end_point(r, o)
    assert r.t_star < -1e-6


@pytest.mark.parametrize("dp,d", [(1, 1), (2, 2)])
def test_scalar_unstable_vertex(P, dp, d):
    """n = 1 is a linear program: a certificate exists iff every vertex is
    negative; one positive vertex makes it INFEASIBLE at every degree."""
    A = np.array([[[-0.5]], [[0.3]], [[-2.0]]])
    g = P.polya_setup(A, 1, 3, dp, d)
    r = P.ipm_solve(g)
    o = ipm.ipm_solve(S.make_sdp(A, 1, 3, dp, d))
    assert o.verdict == ipm.INFEASIBLE
    assert r.verdict == P.INFEASIBLE, (r.reason_name, r.t_star)
    assert r.verdict == o.verdict and r.phase1_used == o.phase1_used


@pytest.mark.parametrize("a", [0.2, 2.0])
def test_paper_literal_absolute_gap(P, a):
    """The paper as printed: C_j = 0 on derivative blocks and the absolute gap
    test alone.  A_i = -aI: the optimum is l^dp n delta."""
    n, l, dp, d = 3, 3, 1, 1
    A = np.repeat((-a * np.eye(n))[None], l, axis=0)
    g = P.polya_setup(A, n, l, dp, d, paper_literal=True)
    assert np.all(g.get_polya()["cdiag"][g.L:] == 0.0)
    o = ipm.ipm_solve(S.make_sdp(A, n, l, dp, d, paper_literal=True), ipm.Options(stop_rule="absolute"))
    r = P.ipm_solve(g, stop_rule="absolute")
    want = l ** dp * n * 1e-3
    assert r.verdict == P.FEASIBLE and r.gap_abs <= 1e-8
    assert abs(r.psi - want) <= 1e-8 + 1e-6 * want
    _same_end_point(r, o, margin="margin_P")


@pytest.mark.parametrize("seed", [0, 1, 2, 5])
def test_paper_literal_seeds(P, seed):
    sy = W.plain_system(seed)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d, paper_literal=True)
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d, paper_literal=True))
    r = P.ipm_solve(g)
    # with C_j = 0 the derivative blocks carry no margin of their own: their
    # lambda_min is not fixed by the optimum, the P-block margin is (delta)
    _same_end_point(r, o, margin="margin_P")
    assert r.margin > 0
    ra = P.ipm_solve(g, stop_rule="absolute")
    oa = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d, paper_literal=True),
                       ipm.Options(stop_rule="absolute"))
    assert ra.verdict == oa.verdict
    assert abs(ra.iterations - oa.iterations) <= 1
    if oa.verdict == ipm.FEASIBLE:
        assert ra.gap_abs <= 1e-8
        assert abs(ra.psi - oa.psi) <= 1e-8 + 1e-6 * abs(oa.psi)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_mehrotra_sigma(P, seed):
    _flush(f"mehrotra seed={seed}")
    sy = W.plain_system(seed)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r = P.ipm_solve(g, sigma_rule="mehrotra")
    o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(sigma_rule="mehrotra"))
    _same_end_point(r, o)
    r0 = P.ipm_solve(g)
    assert r.iterations <= r0.iterations


def test_mehrotra_n10_batch(P):
    """Mehrotra's sigma over a batch of the n = 10 family (small-block fused
    kernels) and one twin (phase-I): the oracle's end points."""
    sys_ = [W.c1_system(s) for s in range(4)] + [W.plain_system(2, twin=True)]
    gs = [P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d) for sy in sys_]
    _flush("mehrotra batch")
    rb = P.ipm_solve_batched(gs, sigma_rule="mehrotra")
    for sy, r in zip(sys_, rb):
        o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d), ipm.Options(sigma_rule="mehrotra"))
        _same_end_point(r, o)

"""The allocation-free solve (psdp_ipm_solve_noalloc) against the allocating
one (psdp_ipm_solve), both through the C ABI (marker: gpu).

Both run the same kernels on the same kernel paths, so the results must be
identical: verdict, exit reason, iteration counts and the dual vector bit for
bit.  Two calls in a row share the library's static scratch, the second on a
smaller system (and a third on a system that needs phase-I); the end points
are also checked against the FP64 oracle.  A system whose solve does not fit
the scratch is rejected before any device work.
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


def _paths(g):
    # the default kernel paths, named explicitly so that the allocating solve
    # does not pick others through its autotuner
    return dict(asm_path=1 if g.n * g.n <= 128 else 0, solve_path=1 if g.Kpad // 64 <= 32 else 0)


def _same(r0, r1):
    assert r1.verdict == r0.verdict and r1.reason == r0.reason
    assert r1.iterations == r0.iterations
    assert r1.phase1_used == r0.phase1_used and r1.phase1_iterations == r0.phase1_iterations
    assert np.array_equal(r1.y, r0.y)
    assert np.array_equal(r1.P, r0.P)
    for k in ("psi", "phi", "margin", "t_star"):
        a, b = getattr(r0, k), getattr(r1, k)
        assert (a == b) or (a != a and b != b), (k, a, b)
    assert r1.graph_replays == 0


@pytest.mark.parametrize("order", ["large_first", "small_first"])
def test_noalloc_equals_solve(P, order):
    cases = [W.c1_system(3), W.plain_system(2), W.plain_system(1, twin=True)]
    if order == "small_first":
        cases = cases[1:] + cases[:1]
    for sy in cases:
        print(f"noalloc {sy.tag} seed={sy.seed}", flush=True)
        g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
        r0 = P.ipm_solve(g, **_paths(g))
        r1 = P.ipm_solve_noalloc(g, **_paths(g))
        _same(r0, r1)
        o = ipm.ipm_solve(S.make_sdp(sy.A, sy.n, sy.l, sy.dp, sy.d))
        assert r1.verdict == o.verdict
        if o.verdict == ipm.FEASIBLE:
            assert abs(r1.psi - o.psi) <= 1e-6 * abs(o.psi)
            assert abs(r1.margin - o.margin) <= 1e-6 * abs(o.margin)


def test_noalloc_precision_form(P):
    sy = W.c1_system(5)
    g = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    r0 = P.ipm_solve(g, precision="fp32", **_paths(g))
    r1 = P.ipm_solve_noalloc(g, precision="fp32", **_paths(g))
    _same(r0, r1)
    assert r1.iters_lowprec == r0.iters_lowprec and r1.ir_steps == r0.ir_steps


def test_noalloc_rejects_too_large(P):
    """K = 6240: the Schur matrix alone (8 Kpad^2 bytes, 311 MB) exceeds the
    scratch; the call fails with EINVAL and a later small call still works."""
    A = W.dissip_vertices(0, 64, 3, 0.3)
    g = P.polya_setup(A, 64, 3, 1, 1)
    with pytest.raises(P.PsdpError) as ei:
        P.ipm_solve_noalloc(g)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    sy = W.plain_system(0)
    g2 = P.polya_setup(sy.A, sy.n, sy.l, sy.dp, sy.d)
    _same(P.ipm_solve(g2, **_paths(g2)), P.ipm_solve_noalloc(g2, **_paths(g2)))

"""Predictor-corrector primal-dual interior-point method (oracle).  Test
infrastructure only.

Follows Section IV-A and Alg. 2 of the paper:

    primal  max tr(CX)  s.t. B(X) = a, X >= 0
    dual    min a^T y   s.t. B^T(y) - C = Z >= 0

with, per iteration (all matrices block-diagonal, Theorem 3):

    G      = C - B^T(y) + Z                               (eq. G)
    Omega  = [B(Z^-1 B^T(e_l) X)]_l                       (Schur complement)
    dy^    = Omega^-1 (B(Z^-1 G X) - a)                   (predictor)
    dZ^    = -G + B^T(dy^)                                (eq. delZ_hat)
    dX^    = -X - Z^-1 dZ^ X                              (reading of eq. delX_hat)
    mu     = sigma tr(ZX) / m                             (reading: normalised)
    dy-    = Omega^-1 (B(mu Z^-1) - B(Z^-1 dZ^ dX^))      (corrector)
    dZ-    = B^T(dy-)                                     (eq. delz_bar)
    dX-    = mu Z^-1 - Z^-1 dZ^ dX^ - Z^-1 dZ- X          (eq. delx_bar)
    dX     = sym(dX^ + dX-), dZ = dZ^ + dZ-, dy = dy^ + dy-
    X += t_p dX,  Z += t_d dZ,  y += t_d dy                (eq. X, y, Z)

Readings where the paper is silent or garbled (each is listed in the design
notes): eq. delX_hat prints a product G B^T(dy) that is inconsistent with the
predictor equation; the form above is the one that gives B(X + dX^) = a.  mu is
printed as tr(ZX)/3 without the 1/m normalisation; the normalised form is used.
dX is symmetrised.  The line search is "standard": a geometric ladder of trial
steps tested by block Cholesky.  The stopping rule is a scale-relative gap plus
primal and dual residuals.  Options give the paper's own forms as modes: the
absolute gap test alone (stop_rule="absolute"; with paper_literal set-up,
whose derivative blocks have C_j = 0, this is the paper as printed), and
Mehrotra's adaptive sigma in place of the fixed 1/3.

The iteration trajectory itself is parity unpinned (rounding at the Cholesky
boundary of the ladder can shift an iteration); the end points are pinned by
closed forms in the tests.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np

from .sdp import PolyaSDP, schur_expanded

FEASIBLE, INFEASIBLE, UNKNOWN = 0, 1, 2
VERDICT_NAMES = {FEASIBLE: "FEASIBLE", INFEASIBLE: "INFEASIBLE", UNKNOWN: "UNKNOWN"}

# exit reasons of one IPM run
CONVERGED, FARKAS, STALL, MAXITER, LADDER_FAIL, CHOL_FAIL, NONFINITE = range(7)
REASON_NAMES = ["converged", "farkas", "stall", "max_iter", "ladder_fail", "chol_fail", "nonfinite"]


@dataclass
class Options:
    gap_tol: float = 1e-8
    feas_tol: float = 1e-8
    max_iter: int = 100
    sigma: float = 1.0 / 3.0
    step_frac: float = 0.95
    ladder_rho: float = 0.9
    ladder_len: int = 300
    farkas_tol: float = 1e-6
    stall_window: int = 10
    stall_drop: float = 0.1
    shift_first: float = 1e-14
    shift_growth: float = 100.0
    shift_max: float = 1e-6
    ir_steps: int = 2
    shift_force: float = 0.0      # > 0: every Schur factorisation starts shifted by this x max diag
    phase1_tol: float = 1e-6
    verdict_mode: str = "paper_then_phase1"   # or "paper_only", "phase1_only"
    stop_rule: str = "relative"   # or "absolute": the paper's |a^T y - tr(CX)| <= gap_tol alone
    sigma_rule: str = "fixed"     # or "mehrotra": sigma = (mu_aff / mu)^3 from the predictor step


# ---------------------------------------------------------------------------
# block linear algebra helpers
# ---------------------------------------------------------------------------

def chol_ok(Mb: np.ndarray) -> bool:
    try:
        np.linalg.cholesky(Mb)
        return True
    except np.linalg.LinAlgError:
        return False


def block_inverse(Z: np.ndarray) -> np.ndarray:
    """Z_j^{-1} through the Cholesky factor of each block."""
    out = np.empty_like(Z)
    I = np.eye(Z.shape[1])
    for j in range(Z.shape[0]):
        R = np.linalg.cholesky(Z[j])
        Linv = np.linalg.solve(R, I)
        out[j] = Linv.T @ Linv
    return out


def ladder(V: np.ndarray, dV: np.ndarray, opt: Options) -> Optional[float]:
    """Step length rule (reading of "a standard line-search ... with the
    constraint that X and Z remain positive semidefinite"): with
    r_0 = 1, r_{k+1} = 0.9 r_k (repeated multiplication), the trial steps are
    T_k = r_k / 0.95 for k = 0..ladder_len.  Per block, k_j is the first k at
    which V_j + T_k dV_j passes Cholesky; with k* = max_j k_j the step is
    0.95 T_{k*} = r_{k*}.  None if some block never passes."""
    rs = [1.0]
    for _ in range(opt.ladder_len):
        rs.append(rs[-1] * opt.ladder_rho)
    kmax = 0
    for j in range(V.shape[0]):
        ok = False
        for k in range(opt.ladder_len + 1):
            if chol_ok(V[j] + (rs[k] / opt.step_frac) * dV[j]):
                kmax = max(kmax, k)
                ok = True
                break
        if not ok:
            return None
    return rs[kmax]


# ---------------------------------------------------------------------------
# SDP operator bundles: the paper's SDP and the phase-I margin SDP
# ---------------------------------------------------------------------------

class PaperOps:
    """The SDP of Section III-B."""

    def __init__(self, sdp: PolyaSDP):
        self.sdp = sdp
        self.K = sdp.K
        self.n = sdp.bn
        self.nb = sdp.nb
        self.C = sdp.C_blocks()
        self.a = sdp.a()

    def BT(self, y):
        return self.sdp.BT(y)

    def B(self, W):
        return self.sdp.B(W)

    def schur(self, X, Zi):
        return self.sdp.schur(X, Zi)

    def init_y(self):
        return np.zeros(self.K)


class Phase1Ops:
    """Phase-I margin SDP (an addition to the paper, which has no
    infeasibility mechanism):  max t  s.t.  B^T(y) - t D >= 0,  a^T y = 1,
    with D = diag(s_j I) built from the multinomial block scales.  The
    equality is removed by eliminating the last entry of y:
    y = (u, 1 - sum u), so the unknowns are (u, t) in R^K and
        F_i = B_i - B_K (i < K),  F_t = -D,  F_0 = -B_K,  objective min -t.
    Its Schur complement follows from the paper's one:
        L'_ij = L_ij - L_iK - L_Kj + L_KK,
        L'_it = -(v_i - v_K) with v = B(Z^-1 D X),
        L'_tt = tr(D Z^-1 D X)."""

    def __init__(self, sdp: PolyaSDP):
        self.sdp = sdp
        self.K = sdp.K
        self.n = sdp.bn
        self.nb = sdp.nb
        self.D = sdp.scale
        eK = np.zeros(sdp.K)
        eK[-1] = 1.0
        self.C = -sdp.BT(eK)
        self.a = np.zeros(sdp.K)
        self.a[-1] = -1.0

    def lift(self, yp):
        """Linear part: u -> (u, -sum u); the t entry is handled apart."""
        y = np.empty(self.K)
        y[:-1] = yp[:-1]
        y[-1] = -np.sum(yp[:-1])
        return y

    def full_y(self, yp):
        """The actual y of the paper's SDP, with a^T y = 1."""
        y = self.lift(yp)
        y[-1] += 1.0
        return y

    def BT(self, yp):
        out = self.sdp.BT(self.lift(yp))
        out -= yp[-1] * self.D[:, None, None] * np.eye(self.n)[None]
        return out

    def B(self, W):
        b = self.sdp.B(W)
        out = np.empty(self.K)
        out[:-1] = b[:-1] - b[-1]
        out[-1] = -np.sum(self.D * np.trace(W, axis1=1, axis2=2))
        return out

    def schur(self, X, Zi):
        Lm = self.sdp.schur(X, Zi)
        K = self.K
        out = np.empty((K, K))
        out[:-1, :-1] = Lm[:-1, :-1] - Lm[:-1, -1:] - Lm[-1:, :-1] + Lm[-1, -1]
        W = self.D[:, None, None] * np.einsum("jab,jbc->jac", Zi, X)
        v = self.sdp.B(W)
        out[:-1, -1] = -(v[:-1] - v[-1])
        out[-1, :-1] = out[:-1, -1]
        out[-1, -1] = np.sum(self.D ** 2 * np.einsum("jab,jba->j", Zi, X))
        return out

    def init_y(self):
        yp = np.full(self.K, 1.0 / self.K)
        yp[-1] = 0.0
        return yp


# ---------------------------------------------------------------------------
# one IPM run
# ---------------------------------------------------------------------------

@dataclass
class RunResult:
    reason: int
    iterations: int
    X: np.ndarray
    Z: np.ndarray
    y: np.ndarray
    phi: float
    psi: float
    gap_abs: float
    gap_rel: float
    pinf: float
    dinf: float
    history: List[dict] = field(default_factory=list)
    shifts: int = 0


def _factor_with_shift(Lam: np.ndarray, opt: Options):
    """Cholesky of the Schur matrix (Alg. 2, root step 1).  The paper assumes
    it succeeds; near the optimum the matrix is so ill-conditioned that a
    pivot can turn non-positive by rounding.  Then the factorisation is
    retried with a diagonal shift tau = shift_first * max diag, growing
    x shift_growth while tau <= shift_max * max diag; the first success is
    kept.  With shift_force > 0 the unshifted attempt is skipped and the
    first shift is shift_force * max diag.  Returns (R, tau) or (None, None)."""
    if opt.shift_force <= 0.0:
        try:
            return np.linalg.cholesky(Lam), 0.0
        except np.linalg.LinAlgError:
            pass
    dmax = float(np.max(np.diag(Lam)))
    tau = (opt.shift_force if opt.shift_force > 0.0 else opt.shift_first) * dmax
    while tau <= opt.shift_max * dmax * (1 + 1e-12):
        try:
            return np.linalg.cholesky(Lam + tau * np.eye(Lam.shape[0])), tau
        except np.linalg.LinAlgError:
            tau *= opt.shift_growth
    return None, None


def _solve(R: np.ndarray, tau: float, Lam: np.ndarray, rhs: np.ndarray, opt: Options) -> np.ndarray:
    """Newton solve with the factor R of Lam + tau I; when tau > 0, ir_steps
    corrections x += (R R^T)^{-1} (rhs - Lam x) against the unshifted Lam."""
    from scipy.linalg import solve_triangular
    def s(b):
        z = solve_triangular(R, b, lower=True)
        return solve_triangular(R.T, z, lower=False)
    x = s(rhs)
    if tau > 0.0:
        for _ in range(opt.ir_steps):                    # refine against the unshifted matrix
            x = x + s(rhs - Lam @ x)
    return x


def ipm_run(ops, opt: Options, phase1: bool = False,
            callback: Optional[Callable] = None, start=None, max_iter: Optional[int] = None) -> RunResult:
    n, nb, K = ops.n, ops.nb, ops.K
    m = nb * n
    I = np.eye(n)
    X = np.repeat(I[None], nb, axis=0)
    Z = X.copy()
    y = ops.init_y()
    if start is not None:
        X, y, Z = (np.array(v, dtype=np.float64, copy=True) for v in start)
    cap = opt.max_iter if max_iter is None else max_iter
    a = ops.a
    C = ops.C
    normC = np.linalg.norm(C)
    norma = np.linalg.norm(a)
    hist: List[dict] = []
    reason = MAXITER
    shifts = 0
    it = 0
    phi = psi = gap_abs = gap_rel = pinf = dinf = float("nan")
    while True:
        try:
            Zi = block_inverse(Z)
        except np.linalg.LinAlgError:
            # a block of Z lost definiteness by rounding: the run ends as
            # non-finite (its last scalars stay those of the previous pass)
            reason = NONFINITE
            break
        G = C - ops.BT(y) + Z
        BX = ops.B(X)
        phi = float(np.sum(np.einsum("jab,jba->j", C, X)))
        psi = float(a @ y)
        trZX = float(np.sum(np.einsum("jab,jba->j", Z, X)))
        pinf = float(np.linalg.norm(BX - a) / (1.0 + norma))
        dinf = float(np.linalg.norm(G) / (1.0 + normC))
        gap_abs = abs(psi - phi)
        den = max(abs(psi), abs(phi))
        gap_rel = gap_abs / den if den > 0 else gap_abs
        rec = dict(it=it, phi=phi, psi=psi, gap_rel=gap_rel, pinf=pinf, dinf=dinf, trZX=trZX)
        hist.append(rec)
        if callback:
            callback(rec)
        if not all(np.isfinite([phi, psi, pinf, dinf, trZX])):
            reason = NONFINITE
            break
        if opt.stop_rule == "absolute" and not phase1:
            # the paper's stopping test (Section IV-A): the absolute duality
            # gap alone, with no feasibility test
            if gap_abs <= opt.gap_tol:
                reason = CONVERGED
                break
        else:
            gap_ok = gap_rel <= opt.gap_tol or (phase1 and gap_abs <= 1e-2 * opt.gap_tol)
            if gap_ok and pinf <= opt.feas_tol and dinf <= opt.feas_tol:
                reason = CONVERGED
                break
        if not phase1:
            if phi > 0 and np.linalg.norm(BX) / phi <= opt.farkas_tol:
                reason = FARKAS
                break
            # stall: the dual residual, still above tolerance, has not fallen
            # by 10x over the last stall_window iterations
            w = opt.stall_window
            if it >= w and dinf > opt.feas_tol and dinf > opt.stall_drop * hist[it - w]["dinf"]:
                reason = STALL
                break
        if it >= cap:
            reason = MAXITER
            break
        # Newton system
        Lam = ops.schur(X, Zi)
        R, tau = _factor_with_shift(Lam, opt)
        if R is None:
            reason = CHOL_FAIL
            break
        if tau > 0:
            shifts += 1
        ZiGX = np.einsum("jab,jbc,jcd->jad", Zi, G, X)
        dyh = _solve(R, tau, Lam, ops.B(ZiGX) - a, opt)
        dZh = -G + ops.BT(dyh)
        dXh = -X - np.einsum("jab,jbc,jcd->jad", Zi, dZh, X)
        sigma = opt.sigma
        if opt.sigma_rule == "mehrotra":
            # Mehrotra's heuristic: the predictor step's own step lengths give
            # mu_aff = tr((Z + td dZ^)(X + tp dX^)) / m and sigma = (mu_aff / mu)^3
            # (clipped to [0, 1]); if either ladder fails the fixed sigma stays
            tpa = ladder(X, 0.5 * (dXh + np.transpose(dXh, (0, 2, 1))), opt)
            tda = ladder(Z, dZh, opt)
            if tpa is not None and tda is not None:
                mu_aff = float(np.sum(np.einsum("jab,jba->j", Z + tda * dZh, X + tpa * dXh))) / m
                sigma = min(1.0, max(0.0, (mu_aff / (trZX / m)) ** 3))
        mu = sigma * trZX / m
        Wc = mu * Zi - np.einsum("jab,jbc,jcd->jad", Zi, dZh, dXh)
        dyb = _solve(R, tau, Lam, ops.B(Wc), opt)
        dZb = ops.BT(dyb)
        dXb = Wc - np.einsum("jab,jbc,jcd->jad", Zi, dZb, X)
        dX = dXh + dXb
        dX = 0.5 * (dX + np.transpose(dX, (0, 2, 1)))
        dZ = dZh + dZb
        dy = dyh + dyb
        tp = ladder(X, dX, opt)
        td = ladder(Z, dZ, opt)
        if tp is None or td is None:
            reason = LADDER_FAIL
            break
        X = X + tp * dX
        Z = Z + td * dZ
        y = y + td * dy
        hist[-1].update(mu=mu, tp=tp, td=td)
        it += 1
    return RunResult(reason, it, X, Z, y, phi, psi, gap_abs, gap_rel, pinf, dinf, hist, shifts)


# ---------------------------------------------------------------------------
# certificate (Alg. 2 final root step, plus an explicit check)
# ---------------------------------------------------------------------------

def certificate(sdp: PolyaSDP, y: np.ndarray):
    """Q_j = B^T(y)_j recomputed from y; passes iff every block factors;
    margin = min_j lambda_min(Q_j) / s_j with s_j the block's multinomial
    scale.  Returns (passes, margin, margin_P, margin_D)."""
    Q = sdp.BT(y)
    ok = all(chol_ok(Q[j]) for j in range(sdp.nb))
    lm = np.array([np.linalg.eigvalsh(Q[j])[0] for j in range(sdp.nb)]) / sdp.scale
    return ok, float(lm.min()), float(lm[:sdp.L].min()), float(lm[sdp.L:].min())


@dataclass
class SolveResult:
    verdict: int
    P: np.ndarray
    y: np.ndarray
    phi: float
    psi: float
    gap_abs: float
    gap_rel: float
    pinf: float
    dinf: float
    margin: float
    margin_P: float
    margin_D: float
    iterations: int
    reason: int
    chol_shifts: int = 0          # iterations whose Schur factorisation needed a shift
    phase1_used: bool = False
    phase1_iterations: int = 0
    phase1_reason: int = -1
    t_star: float = float("nan")
    warm_used: bool = False
    warm_fallback: bool = False
    warm_iterations: int = 0


def warm_start_point(sdp: PolyaSDP, y0: np.ndarray, logx: Optional[np.ndarray] = None,
                     margin: float = 1e-6, center: bool = True):
    """Interior starting point from a predicted dual vector y0 and predicted
    log block scales s_j of X (learned warm start; not part of the paper).

    Z_j = B^T(y0)_j - C_j + tau_j I with tau_j = max(0, margin s'_j -
    lambda_min(B^T(y0)_j - C_j)) (s'_j the block scale), so that Z_j >=
    margin s'_j I; X_j = exp(s_j) n Z_j^{-1} / tr(Z_j^{-1}) (center) or
    exp(s_j) I.  lambda_min is taken from the symmetric eigensolver."""
    nb, n = sdp.nb, sdp.bn
    s = np.zeros(nb) if logx is None else np.asarray(logx, dtype=np.float64)
    W = sdp.BT(np.asarray(y0, dtype=np.float64)) - sdp.C_blocks()
    X = np.empty_like(W)
    Z = np.empty_like(W)
    I = np.eye(n)
    for j in range(nb):
        lam = float(np.linalg.eigvalsh(W[j])[0])
        tau = max(0.0, margin * sdp.scale[j] - lam)
        Z[j] = W[j] + tau * I
        if center:
            Zi = np.linalg.inv(Z[j])
            Zi = 0.5 * (Zi + Zi.T)
            X[j] = np.exp(s[j]) * n * Zi / np.trace(Zi)
        else:
            X[j] = np.exp(s[j]) * I
    return X, np.array(y0, dtype=np.float64), Z


def ipm_solve(sdp: PolyaSDP, opt: Optional[Options] = None, warm=None,
              warm_iter_cap: int = 0, warm_margin: float = 1e-6,
              warm_center: bool = True) -> SolveResult:
    """With warm = (y0, logx): the paper's SDP is first solved from
    warm_start_point (at most warm_iter_cap iterations, 0: max_iter); a
    converged run with a passing certificate gives FEASIBLE and a Farkas ray
    INFEASIBLE; anything else falls back to the cold pipeline below.
    SolveResult.warm_used / warm_fallback / warm_iterations record which."""
    opt = opt or Options()
    if warm is not None:
        start = warm_start_point(sdp, warm[0], warm[1], warm_margin, warm_center)
        cap = warm_iter_cap if warm_iter_cap > 0 else opt.max_iter
        r = ipm_run(PaperOps(sdp), opt, start=start, max_iter=min(cap, opt.max_iter))
        if r.reason == CONVERGED:
            ok, mg, mP, mD = certificate(sdp, r.y)
            if ok:
                res = SolveResult(FEASIBLE, sdp.P_of_y(r.y), r.y, r.phi, r.psi, r.gap_abs, r.gap_rel,
                                  r.pinf, r.dinf, mg, mP, mD, r.iterations, r.reason, r.shifts)
                res.warm_used, res.warm_iterations = True, r.iterations
                return res
        elif r.reason == FARKAS:
            nanv = float("nan")
            res = SolveResult(INFEASIBLE, np.zeros((sdp.L0, sdp.pn, sdp.pn)), r.y, r.phi, r.psi,
                              r.gap_abs, r.gap_rel, r.pinf, r.dinf, nanv, nanv, nanv, r.iterations,
                              r.reason)
            res.warm_used, res.warm_iterations = True, r.iterations
            return res
        res = ipm_solve(sdp, opt)
        res.warm_fallback, res.warm_iterations = True, r.iterations
        return res
    return _solve_cold(sdp, opt)


def _solve_cold(sdp: PolyaSDP, opt: Options) -> SolveResult:
    """Verdict pipeline: the paper's SDP first; FEASIBLE when it converges and
    the certificate check passes; INFEASIBLE on a Farkas ray; otherwise the
    phase-I margin SDP decides by the sign of t* (|t*| <= phase1_tol gives
    UNKNOWN)."""
    opt = opt or Options()
    nanv = float("nan")
    zeroP = np.zeros((sdp.L0, sdp.pn, sdp.pn))
    if opt.verdict_mode != "phase1_only":
        r = ipm_run(PaperOps(sdp), opt)
        if r.reason == CONVERGED:
            ok, mg, mP, mD = certificate(sdp, r.y)
            verdict = FEASIBLE if ok else UNKNOWN
            return SolveResult(verdict, sdp.P_of_y(r.y), r.y, r.phi, r.psi, r.gap_abs, r.gap_rel,
                               r.pinf, r.dinf, mg, mP, mD, r.iterations, r.reason, r.shifts)
        if r.reason == FARKAS or opt.verdict_mode == "paper_only":
            v = INFEASIBLE if r.reason == FARKAS else UNKNOWN
            return SolveResult(v, zeroP, r.y, r.phi, r.psi, r.gap_abs, r.gap_rel, r.pinf, r.dinf,
                               nanv, nanv, nanv, r.iterations, r.reason, r.shifts)
        its, reason0, shifts0 = r.iterations, r.reason, r.shifts
    else:
        its, reason0, shifts0 = 0, -1, 0
    p1 = Phase1Ops(sdp)
    r1 = ipm_run(p1, opt, phase1=True)
    t = float(r1.y[-1])
    decided = r1.reason == CONVERGED or (
        r1.reason == CHOL_FAIL and abs(t) > r1.gap_abs and r1.pinf <= 1e-6 and r1.dinf <= 1e-6)
    if decided and t > opt.phase1_tol:
        yfull = p1.full_y(r1.y)
        # rescale the margin certificate onto the paper's constraint B^T(y) >= C
        ratio = np.max(sdp.cdiag / sdp.scale) / t
        ycert = yfull * ratio
        ok, mg, mP, mD = certificate(sdp, ycert)
        verdict = FEASIBLE if ok else UNKNOWN
        res = SolveResult(verdict, sdp.P_of_y(ycert), ycert, nanv, float(np.sum(ycert)), nanv, nanv,
                          r1.pinf, r1.dinf, mg, mP, mD, its, reason0)
    elif decided and t < -opt.phase1_tol:
        res = SolveResult(INFEASIBLE, zeroP, p1.full_y(r1.y), nanv, nanv, nanv, nanv, r1.pinf, r1.dinf,
                          nanv, nanv, nanv, its, reason0)
    else:
        res = SolveResult(UNKNOWN, zeroP, p1.full_y(r1.y), nanv, nanv, nanv, nanv, r1.pinf, r1.dinf,
                          nanv, nanv, nanv, its, reason0)
    res.chol_shifts = shifts0 + r1.shifts
    res.phase1_used = True
    res.phase1_iterations = r1.iterations
    res.phase1_reason = r1.reason
    res.t_star = t
    return res


# ---------------------------------------------------------------------------
# dense textbook primal-dual method on the full (L+M)n matrices (Theorem 3)
# ---------------------------------------------------------------------------

def dense_ipm(sdp: PolyaSDP, opt: Optional[Options] = None, iters: int = 60):
    """The same predictor-corrector steps written on dense matrices with every
    B_k materialised (tiny problems only).  Used to check Theorem 3: started
    from block-diagonal X, Z the off-block entries stay exactly zero, and the
    objective equals the block method's.  Returns (X, Z, y, history)."""
    opt = opt or Options()
    mdim = sdp.m
    Bs = [sdp.dense_B(k) for k in range(sdp.K)]
    C = sdp.dense_C()
    a = sdp.a()
    X = np.eye(mdim)
    Z = np.eye(mdim)
    y = np.zeros(sdp.K)

    def BT(v):
        return sum(v[k] * Bs[k] for k in range(sdp.K))

    def Bop(W):
        return np.array([np.trace(Bk @ W) for Bk in Bs])

    def step(V, dV):
        r = 1.0
        for k in range(opt.ladder_len + 1):
            if chol_ok(V + (r / opt.step_frac) * dV):
                return r
            r *= opt.ladder_rho
        return None

    hist = []
    for it in range(iters):
        Zi = np.linalg.inv(Z)
        G = C - BT(y) + Z
        phi, psi = float(np.trace(C @ X)), float(a @ y)
        hist.append(dict(phi=phi, psi=psi))
        if abs(psi - phi) <= opt.gap_tol * max(abs(psi), abs(phi)) and \
                np.linalg.norm(Bop(X) - a) <= opt.feas_tol * (1 + np.linalg.norm(a)):
            break
        Lam = np.array([[np.trace(Bs[k] @ Zi @ Bs[l] @ X) for l in range(sdp.K)] for k in range(sdp.K)])
        dyh = np.linalg.solve(Lam, Bop(Zi @ G @ X) - a)
        dZh = -G + BT(dyh)
        dXh = -X - Zi @ dZh @ X
        mu = opt.sigma * np.trace(Z @ X) / mdim
        Wc = mu * Zi - Zi @ dZh @ dXh
        dyb = np.linalg.solve(Lam, Bop(Wc))
        dZb = BT(dyb)
        dXb = Wc - Zi @ dZb @ X
        dX = dXh + dXb
        dX = 0.5 * (dX + dX.T)
        tp, td = step(X, dX), step(Z, dZh + dZb)
        X = X + tp * dX
        Z = Z + td * (dZh + dZb)
        y = y + td * (dyh + dyb)
    return X, Z, y, hist

"""Robust-stability radius by bisection over translated simplices (oracle).
Test infrastructure only: the FP64 reference of the library's
psdp_poly_on_simplex and psdp_bisect_simplex, never imported by the product.

Section II turns a non-homogeneous A(alpha) on the simplex into a homogeneous
one by multiplying each monomial of degree k by (sum alpha)^(da-k).  Section
V (Examples 1 and 2) studies regions that are simplices translated away from
the unit one: the uncertain parameter x lies in the image of Delta_l under a
linear map x = G alpha, and A(G alpha) is again a polynomial in alpha.  With
both steps the system on the region becomes a homogeneous A'(alpha) on
Delta_l, whose certificate by the Polya SDP proves stability on the region.
The examples then bisect the size of the region.

Readings (where the text is ambiguous):
* Example 2 says its map is "as in Example 1", but that map sends Delta_3 onto
  a set with coordinate sum -|rho|, not onto S_L = {sum x = 2L + 1,
  L <= x_i <= 1}.  The homogeneous map g_i(alpha) = L sum_j alpha_j +
  (1 - L) alpha_i does map Delta_3 onto S_L (vertex e_i goes to the point with
  x_i = 1 and the others L), so G(L) = I + L (11^T - I).
* Example 1's map g_i = 2|rho| (alpha_i - 1/2) has a constant term; on the
  simplex 1/2 = (1/2) sum_j alpha_j, which makes it linear:
  G(rho) = rho (2 I - 11^T), sending Delta_l onto the translated simplex with
  coordinate sum -(l - 2) rho and |x_i| <= rho (the text's S_rho for l = 8).
* Only a certified (FEASIBLE) verdict moves the bisection's feasible end; an
  UNKNOWN counts as no certificate.

Everything here is a plain expansion: monomials as exponent tuples,
polynomial products term by term, sums in the order the terms are listed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence, Tuple

import numpy as np

from . import ipm, polya, sdp as S

Mono = Tuple[int, ...]


def _mul(p: Dict[Mono, float], q: Dict[Mono, float]) -> Dict[Mono, float]:
    out: Dict[Mono, float] = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0.0) + ca * cb
    return out


def linear_form(G: np.ndarray, i: int) -> Dict[Mono, float]:
    """x_i = sum_j G[i][j] alpha_j as a polynomial in alpha."""
    l = G.shape[1]
    out: Dict[Mono, float] = {}
    for j in range(l):
        e = tuple(1 if k == j else 0 for k in range(l))
        out[e] = float(G[i, j])
    return out


def poly_on_simplex(exps: Sequence[Sequence[int]], mats: np.ndarray, G: np.ndarray | None,
                    l: int, da: int) -> np.ndarray:
    """Coefficients [f(l, da)][n][n] (W_da, descending lex) of
        B(alpha) = sum_t (sum_j alpha_j)^(da - |lam_t|) mats[t] (G alpha)^lam_t,
    which equals A(G alpha) = sum_t mats[t] (G alpha)^lam_t on Delta_l.
    G = None is the identity (plain homogenisation, Section II)."""
    mats = np.asarray(mats, dtype=np.float64)
    n = mats.shape[1]
    if G is None:
        G = np.eye(l)
    G = np.asarray(G, dtype=np.float64)
    W = polya.monomials(l, da)
    idx = polya.index_map(W)
    out = np.zeros((len(W), n, n))
    one = {tuple([0] * l): 1.0}
    for lam, mat in zip(exps, mats):
        k = sum(lam)
        if k > da:
            raise ValueError("a term's degree exceeds da")
        p = dict(one)
        for i, e in enumerate(lam):
            xi = linear_form(G, i)
            for _ in range(e):
                p = _mul(p, xi)
        sp = {m: float(c) for m, c in polya.simplex_power(l, da - k).items()}
        p = _mul(p, sp)
        for m, c in p.items():
            out[idx[m]] = out[idx[m]] + c * mat
    return out


def evaluate(exps, mats, x: np.ndarray) -> np.ndarray:
    """A(x) = sum_t mats[t] x^lam_t."""
    acc = np.zeros(np.asarray(mats).shape[1:])
    for lam, mat in zip(exps, mats):
        acc = acc + float(np.prod([xi ** e for xi, e in zip(x, lam)])) * np.asarray(mat)
    return acc


def evaluate_homogeneous(B: np.ndarray, l: int, da: int, alpha: np.ndarray) -> np.ndarray:
    return sum(float(np.prod(alpha ** np.array(m))) * B[i] for i, m in enumerate(polya.monomials(l, da)))


@dataclass
class BisectResult:
    t_cert: float                 # last value with a certificate (nan: none)
    t_other: float                # the other end of the final bracket
    trials: List[Tuple[float, int, int]] = field(default_factory=list)   # (t, verdict, iterations)


def bisect_simplex(exps, mats, G0: np.ndarray, G1: np.ndarray, l: int, dp: int, d: int,
                   t_feas: float, t_infeas: float, tol: float, opt: ipm.Options | None = None,
                   da: int | None = None, width: int = 1) -> BisectResult:
    """Section V's bisection: the region is the image of Delta_l under
    x = (G0 + t G1) alpha; t moves between t_feas (certificate expected) and
    t_infeas until they are within tol.  t_feas is tried first; each trial
    builds A' = poly_on_simplex(A, G(t)) and solves its Polya SDP at (dp, d).
    A round tries `width` values splitting the bracket evenly (1: the
    midpoint) and keeps the certified ones up to the first that is not."""
    mats = np.asarray(mats, dtype=np.float64)
    n = mats.shape[1]
    da = max(sum(e) for e in exps) if da is None else da
    res = BisectResult(float("nan"), t_infeas)

    def trial(t):
        Ap = poly_on_simplex(exps, mats, G0 + t * G1, l, da)
        r = ipm.ipm_solve(S.make_sdp(Ap, n, l, dp, d, da=da), opt)
        res.trials.append((t, r.verdict, r.iterations + r.phase1_iterations))
        return r.verdict == ipm.FEASIBLE

    if not trial(t_feas):
        return res
    a, b = t_feas, t_infeas
    while abs(a - b) > tol:
        ts = [a + (b - a) * (i + 1) / (width + 1) for i in range(width)]
        ok = [trial(t) for t in ts]
        na, nb = a, b
        for t, f in zip(ts, ok):
            if not f:
                nb = t
                break
            na = t
        a, b = na, nb
    res.t_cert, res.t_other = a, b
    return res


def spectral_boundary(exps, mats, G0, G1, l: int, t_stable: float, t_unstable: float, tol: float,
                      grid: int) -> float:
    """Brute-force counterpart: bisection on t of "A(G(t) alpha) is Hurwitz at
    every point of the simplex grid with spacing 1/grid".  Stability on the
    region implies this grid test, so a certified t can never lie beyond the
    value returned here (up to tol)."""
    pts = [np.array(m, dtype=np.float64) / grid for m in polya.monomials(l, grid)]

    def stable(t):
        G = G0 + t * G1
        for a in pts:
            x = G @ a
            if np.max(np.linalg.eigvals(evaluate(exps, mats, x)).real) >= 0.0:
                return False
        return True

    a, b = t_stable, t_unstable
    while abs(a - b) > tol:
        mid = 0.5 * (a + b)
        if stable(mid):
            a = mid
        else:
            b = mid
    return b


# ---------------------------------------------------------------------------
# Example 2 of Section V: degree-3 A on S_L, minimise L (its six printed
# coefficient matrices are test data, tests/golden/example2_matrices.txt)
# ---------------------------------------------------------------------------

EXAMPLE2_EXPS = [(3, 0, 0), (2, 1, 0), (1, 1, 1), (1, 0, 2), (0, 3, 0), (0, 0, 3)]


def example2_maps(l: int = 3):
    """G(L) = G0 + L G1 with G0 = I and G1 = 11^T - I (reading above)."""
    return np.eye(l), np.ones((l, l)) - np.eye(l)

"""Exact Polya set-up (oracle).  Test infrastructure only.

Everything integer is computed with Python ``int`` (arbitrary precision), so
overflow can only be detected, never suffered.
"""
from __future__ import annotations

from math import comb, factorial
from typing import Dict, List, Sequence, Tuple

import numpy as np

Mono = Tuple[int, ...]


def f(l: int, d: int) -> int:
    """Number of l-variate monomials of degree d (Notation, eq. f)."""
    if l == 0:
        return 0
    return comb(l + d - 1, l - 1)


def monomials(l: int, d: int) -> List[Mono]:
    """W_d in the paper's order (Notation): gamma precedes eta when the first
    nonzero entry of gamma - eta is positive, i.e. descending lexicographic,
    so alpha_1^d comes first."""
    out: List[Mono] = []

    def rec(prefix: List[int], rem: int) -> None:
        if len(prefix) == l - 1:
            out.append(tuple(prefix + [rem]))
            return
        for v in range(rem, -1, -1):
            rec(prefix + [v], rem - v)

    if l <= 0 or d < 0:
        return out
    rec([], d)
    return out


def index_map(mons: Sequence[Mono]) -> Dict[Mono, int]:
    """0-based rank of each exponent in the given ordered list."""
    return {g: i for i, g in enumerate(mons)}


def lex_index_printed(gamma: Sequence[int]) -> int:
    """The index formula exactly as printed in the Notation section (eq. lex),
    1-based.  It enumerates W_d in *ascending* lexicographic order, i.e. the
    reverse of the order the text and the worked examples use; see
    ``lex_index`` for the reading adopted here."""
    l = len(gamma)
    d = sum(gamma)
    tot = 0
    for j in range(1, l):
        s = sum(gamma[: j - 1])
        for i in range(1, gamma[j - 1] + 1):
            tot += f(l - j, d + 1 - s - i)
    return tot + 1


def lex_index(gamma: Sequence[int]) -> int:
    """1-based index in descending lexicographic order: f(l,d) + 1 minus the
    printed formula (reading: the text and the examples fix the order)."""
    return f(len(gamma), sum(gamma)) + 1 - lex_index_printed(gamma)


def multinomial(d: int, parts: Sequence[int]) -> int:
    """d! / prod(parts_i!) for parts summing to d."""
    assert sum(parts) == d and min(parts) >= 0
    out = factorial(d)
    for p in parts:
        out //= factorial(p)
    return out


def _sub(a: Sequence[int], b: Sequence[int]) -> Tuple[int, ...]:
    return tuple(x - y for x, y in zip(a, b))


def _nonneg(a: Sequence[int]) -> bool:
    return all(x >= 0 for x in a)


# ---------------------------------------------------------------------------
# beta coefficients (Section III-A, eq. beta_init and eq. beta)
# ---------------------------------------------------------------------------

def beta_recursion(l: int, dp: int, d1: int) -> List[List[int]]:
    """beta^{(0)}_{h,g} = [h = g] on W_dp; then d1 rounds of
    beta^{(i)}_{h,g} = sum over unit vectors e of beta^{(i-1)}_{h,g-e}
    for g in W_{dp+i}.  Returns [L0][L] Python ints."""
    Wp = monomials(l, dp)
    units = monomials(l, 1)
    rows = []
    for h in Wp:
        cur = {g: (1 if g == h else 0) for g in Wp}
        for i in range(1, d1 + 1):
            nxt = {}
            for g in monomials(l, dp + i):
                acc = 0
                for e in units:
                    ge = _sub(g, e)
                    if _nonneg(ge):
                        acc += cur.get(ge, 0)
                nxt[g] = acc
            cur = nxt
        rows.append([cur[g] for g in monomials(l, dp + d1)])
    return rows


def beta_closed(l: int, dp: int, d1: int) -> List[List[int]]:
    """Closed form: beta_{h,g} = d1! / (g - h)! when g >= h componentwise,
    else 0 (the multinomial coefficient of alpha^{g-h} in (sum alpha)^d1)."""
    out = []
    for h in monomials(l, dp):
        row = []
        for g in monomials(l, dp + d1):
            dg = _sub(g, h)
            row.append(multinomial(d1, dg) if _nonneg(dg) else 0)
        out.append(row)
    return out


def poly_mul(p: Dict[Mono, int], q: Dict[Mono, int]) -> Dict[Mono, int]:
    out: Dict[Mono, int] = {}
    for a, ca in p.items():
        for b, cb in q.items():
            k = tuple(x + y for x, y in zip(a, b))
            out[k] = out.get(k, 0) + ca * cb
    return out


def simplex_power(l: int, d: int) -> Dict[Mono, int]:
    """(alpha_1 + ... + alpha_l)^d expanded by repeated multiplication."""
    one = {tuple([0] * l): 1}
    lin = {e: 1 for e in monomials(l, 1)}
    out = one
    for _ in range(d):
        out = poly_mul(out, lin)
    return out


def beta_bruteforce(l: int, dp: int, d1: int) -> List[List[int]]:
    """Expand (sum alpha)^d1 * alpha^h and read off the coefficients."""
    sp = simplex_power(l, d1)
    out = []
    for h in monomials(l, dp):
        prod = poly_mul(sp, {h: 1})
        out.append([prod.get(g, 0) for g in monomials(l, dp + d1)])
    return out


# ---------------------------------------------------------------------------
# H coefficients (Section III-A, eq. H_init and eq. H).  H is linear in the
# A coefficients, so the recursion is run on integer weights c[h][g][lam]
# with H_{h,g} = sum_lam c[h][g][lam] A_lam.
# ---------------------------------------------------------------------------

def coef_recursion(l: int, dp: int, da: int, d2: int) -> List[List[List[int]]]:
    """c^{(0)}[h][g][lam] = [lam + h = g] on W_{dp+da} (eq. H_init), then d2
    rounds of the unit-vector shift sum (eq. H).  Returns [L0][M][Na]."""
    Wp = monomials(l, dp)
    Wa = monomials(l, da)
    units = monomials(l, 1)
    out = []
    for h in Wp:
        cur = {}
        for g in monomials(l, dp + da):
            cur[g] = [1 if tuple(x + y for x, y in zip(lam, h)) == g else 0 for lam in Wa]
        for i in range(1, d2 + 1):
            nxt = {}
            for g in monomials(l, dp + da + i):
                acc = [0] * len(Wa)
                for e in units:
                    ge = _sub(g, e)
                    if _nonneg(ge) and ge in cur:
                        acc = [a + b for a, b in zip(acc, cur[ge])]
                nxt[g] = acc
            cur = nxt
        out.append([cur[g] for g in monomials(l, dp + da + d2)])
    return out


def coef_closed(l: int, dp: int, da: int, d2: int) -> List[List[List[int]]]:
    """Closed form: c[h][g][lam] = d2! / (g - h - lam)! when nonnegative."""
    out = []
    for h in monomials(l, dp):
        rows = []
        for g in monomials(l, dp + da + d2):
            r = []
            for lam in monomials(l, da):
                dg = _sub(_sub(g, h), lam)
                r.append(multinomial(d2, dg) if _nonneg(dg) else 0)
            rows.append(r)
        out.append(rows)
    return out


def coef_bruteforce(l: int, dp: int, da: int, d2: int) -> List[List[List[int]]]:
    """Expand (sum alpha)^d2 * alpha^h * alpha^lam for every (h, lam)."""
    sp = simplex_power(l, d2)
    Wm = monomials(l, dp + da + d2)
    Wa = monomials(l, da)
    out = []
    for h in monomials(l, dp):
        per_lam = [poly_mul(sp, {tuple(x + y for x, y in zip(h, lam)): 1}) for lam in Wa]
        out.append([[per_lam[k].get(g, 0) for k in range(len(Wa))] for g in Wm])
    return out


def H_from_coef(coef: List[List[List[int]]], A: np.ndarray) -> np.ndarray:
    """H[m][h] = sum_lam c[h][m][lam] * A_lam in FP64, folded left in
    ascending lam index with a separate multiply and add per term (numpy
    does not contract a*b+c).  A is [Na][n][n].  Returns [M][L0][n][n]."""
    L0 = len(coef)
    M = len(coef[0])
    Na, n, _ = A.shape
    H = np.zeros((M, L0, n, n))
    for h in range(L0):
        for m in range(M):
            acc = np.zeros((n, n))
            for lam in range(Na):
                c = coef[h][m][lam]
                if c != 0:
                    acc = acc + float(c) * A[lam]
            H[m, h] = acc
    return H


def homogenize(terms: Dict[Mono, np.ndarray], l: int) -> Dict[Mono, np.ndarray]:
    """Section II: multiply each monomial of degree d_i by (sum alpha)^{da-d_i}
    so that A(alpha) becomes homogeneous of degree da = max d_i."""
    da = max(sum(k) for k in terms)
    out: Dict[Mono, np.ndarray] = {}
    for mono, mat in terms.items():
        sp = simplex_power(l, da - sum(mono))
        for e, c in sp.items():
            g = tuple(x + y for x, y in zip(mono, e))
            out[g] = out.get(g, 0) + c * mat
    return out


def counts(l: int, dp: int, da: int, d1: int, d2: int, n: int) -> dict:
    """L0, L, M (eq. L0, L, M), N~ = n(n+1)/2 and K (eq. K)."""
    L0 = f(l, dp)
    L = f(l, dp + d1)
    M = f(l, dp + da + d2)
    Nt = n * (n + 1) // 2
    return dict(L0=L0, L=L, M=M, Nt=Nt, K=L0 * Nt, nb=L + M, m=(L + M) * n)

"""SDP elements and operators of the Polya LMIs (oracle).  Test infrastructure
only.

Notation follows Section III-B.  Blocks are indexed j = 0..L-1 (the
"P-blocks", one per monomial of W_{dp+d1}) and j = L..L+M-1 (the
"derivative blocks", one per monomial of W_{dp+da+d2}).  The dual variable y
has K = L0 * N~ entries with k = b + N~ * h (eq. K and the map V_h), where b
indexes the basis of the symmetric n x n matrices.

Basis reading: the Notation section defines the diagonal elements and, for
k > n, only the first superdiagonal; it also states that any basis may be
used.  Here: the n diagonal elements E_pp first, then the off-diagonal
elements E_{i,i+s} = e_i e_{i+s}^T + e_{i+s} e_i^T by increasing offset
s = 1..n-1 and row i.  With entries 0/1 the objective a^T y (eq. a) is the
sum of the upper-triangular entries of all P_h.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import factorial
from typing import List

import numpy as np

from . import polya


def basis_pairs(n: int) -> List[tuple]:
    out = [(p, p) for p in range(n)]
    for s in range(1, n):
        for i in range(n - s):
            out.append((i, i + s))
    return out


def vec_to_sym(v: np.ndarray, n: int) -> np.ndarray:
    """V_h restricted to one h: sum_b E_b v_b (eq. V_h)."""
    P = np.zeros((n, n))
    for b, (p, q) in enumerate(basis_pairs(n)):
        P[p, q] = v[b]
        P[q, p] = v[b]
    return P


def basis_matrix(n: int, b: int) -> np.ndarray:
    p, q = basis_pairs(n)[b]
    E = np.zeros((n, n))
    E[p, q] = 1.0
    E[q, p] = 1.0
    return E


def inner_basis(S: np.ndarray, n: int) -> np.ndarray:
    """tr(E_b S) for every basis element b (S need not be symmetric)."""
    pairs = basis_pairs(n)
    out = np.empty(len(pairs))
    for b, (p, q) in enumerate(pairs):
        out[b] = S[p, p] if p == q else S[p, q] + S[q, p]
    return out


@dataclass
class PolyaSDP:
    """The structured SDP of Section III-B for one uncertain system."""

    n: int
    l: int
    dp: int
    da: int
    d1: int
    d2: int
    A: np.ndarray                      # [Na][n][n], coefficients in W_da order
    delta: float = 1e-3
    eps: float = 1e-3
    paper_literal: bool = False
    # filled by build()
    L0: int = 0
    L: int = 0
    M: int = 0
    Nt: int = 0
    K: int = 0
    beta_int: list = field(default_factory=list)
    coef_int: list = field(default_factory=list)
    beta: np.ndarray = None            # [L0][L] float
    H: np.ndarray = None               # [M][L0][n][n]
    scale: np.ndarray = None           # [L+M] multinomial block scales s_j
    cdiag: np.ndarray = None           # [L+M] C_j = cdiag_j * I

    @property
    def nb(self) -> int:
        return self.L + self.M

    @property
    def bn(self) -> int:
        """Order of every block of the SDP."""
        return self.n

    @property
    def pn(self) -> int:
        """Order of the coefficients P_h (the system's n)."""
        return self.n

    @property
    def m(self) -> int:
        return self.nb * self.n

    def build(self) -> "PolyaSDP":
        l, dp, da, d1, d2, n = self.l, self.dp, self.da, self.d1, self.d2, self.n
        cnt = polya.counts(l, dp, da, d1, d2, n)
        self.L0, self.L, self.M, self.Nt, self.K = cnt["L0"], cnt["L"], cnt["M"], cnt["Nt"], cnt["K"]
        self.beta_int = polya.beta_recursion(l, dp, d1)
        self.coef_int = polya.coef_recursion(l, dp, da, d2)
        self.beta = np.array(self.beta_int, dtype=np.float64).reshape(self.L0, self.L)
        self.H = polya.H_from_coef(self.coef_int, np.asarray(self.A, dtype=np.float64))
        Wp = polya.monomials(l, dp)
        WL = polya.monomials(l, dp + d1)
        WM = polya.monomials(l, dp + da + d2)
        # eq. Cj: C_j = delta * I * sum_h beta_{h,j} dp!/h!  (P-blocks)
        sP = []
        for j in range(self.L):
            tot = 0
            for hi, h in enumerate(Wp):
                tot += self.beta_int[hi][j] * polya.multinomial(dp, h)
            sP.append(tot)
        # derivative blocks: the paper sets C_j = 0; the reading used here puts
        # eps times the multinomial of the block's monomial (the coefficient of
        # alpha^gamma in (sum alpha)^{dp+da+d2}), which makes the derivative
        # LMIs strict; paper_literal keeps 0.
        sM = [polya.multinomial(dp + da + d2, g) for g in WM]
        self.scale = np.array(sP + sM, dtype=np.float64)
        eps = 0.0 if self.paper_literal else self.eps
        self.cdiag = np.concatenate([self.delta * np.array(sP, dtype=np.float64),
                                     eps * np.array(sM, dtype=np.float64)])
        self._WL, self._WM, self._Wp = WL, WM, Wp
        return self

    # ------------------------------------------------------------------
    def C_blocks(self) -> np.ndarray:
        return self.cdiag[:, None, None] * np.eye(self.n)[None]

    def a(self) -> np.ndarray:
        return np.ones(self.K)                                  # eq. a

    def P_of_y(self, y: np.ndarray) -> np.ndarray:
        """P_h = V_h(y) for every h (Alg. 2, final root step)."""
        return np.stack([vec_to_sym(y[h * self.Nt:(h + 1) * self.Nt], self.n)
                         for h in range(self.L0)])

    def y_of_P(self, P: np.ndarray) -> np.ndarray:
        pairs = basis_pairs(self.n)
        return np.concatenate([[P[h][p, q] for (p, q) in pairs] for h in range(self.L0)])

    def BT(self, y: np.ndarray) -> np.ndarray:
        """B^T(y) = sum_i y_i B_i (eq. AT), block by block with eq. Aij."""
        P = self.P_of_y(y)
        out = np.zeros((self.nb, self.n, self.n))
        for j in range(self.L):
            for h in range(self.L0):
                if self.beta[h, j] != 0.0:
                    out[j] += self.beta[h, j] * P[h]
        for m in range(self.M):
            acc = np.zeros((self.n, self.n))
            for h in range(self.L0):
                Hm = self.H[m, h]
                acc += Hm.T @ P[h] + P[h] @ Hm
            out[self.L + m] = -acc
        return out

    def B(self, W: np.ndarray) -> np.ndarray:
        """B(W)_k = tr(B_k W) = sum_j tr(B_{k,j} W_j).  For k = (h, b):
        P-blocks give beta_{h,j} tr(E_b W_j); derivative blocks give
        -tr(E_b (W_j H^T + H W_j)) with H = H_{h,j-L}."""
        out = np.zeros(self.K)
        for h in range(self.L0):
            S = np.zeros((self.n, self.n))
            for j in range(self.L):
                if self.beta[h, j] != 0.0:
                    S += self.beta[h, j] * W[j]
            for m in range(self.M):
                Hm = self.H[m, h]
                Wm = W[self.L + m]
                S -= Wm @ Hm.T + Hm @ Wm
            out[h * self.Nt:(h + 1) * self.Nt] = inner_basis(S, self.n)
        return out

    # ------------------------------------------------------------------
    def dense_B(self, k: int) -> np.ndarray:
        """B_k materialised as a dense (L+M)n square matrix from eq. Ai/Aij
        (tiny problems only)."""
        h, b = divmod(k, self.Nt)
        E = basis_matrix(self.n, b)
        n = self.n
        D = np.zeros((self.m, self.m))
        for j in range(self.L):
            D[j * n:(j + 1) * n, j * n:(j + 1) * n] = self.beta[h, j] * E
        for m in range(self.M):
            Hm = self.H[m, h]
            jj = self.L + m
            D[jj * n:(jj + 1) * n, jj * n:(jj + 1) * n] = -(Hm.T @ E + E @ Hm)
        return D

    def dense_C(self) -> np.ndarray:
        return np.diag(np.repeat(self.cdiag, self.n))

    def schur(self, X: np.ndarray, Zi: np.ndarray) -> np.ndarray:
        """The Schur complement (eq. T2) by the expanded Kronecker form."""
        return schur_expanded(self, X, Zi)

    def active_pairs(self, m: int) -> List[int]:
        """h with H_{h,m} not identically zero (gamma_m >= h componentwise)."""
        return [h for h in range(self.L0) if np.any(self.H[m, h] != 0.0)]


def make_sdp(A: np.ndarray, n: int, l: int, dp: int, d: int, *, da: int = 1,
             d1: int | None = None, d2: int | None = None, delta: float = 1e-3,
             eps: float = 1e-3, paper_literal: bool = False) -> PolyaSDP:
    return PolyaSDP(n=n, l=l, dp=dp, da=da, d1=d if d1 is None else d1,
                    d2=d if d2 is None else d2, A=np.asarray(A, dtype=np.float64),
                    delta=delta, eps=eps, paper_literal=paper_literal).build()


def blockdiag(blocks: np.ndarray) -> np.ndarray:
    nb, n, _ = blocks.shape
    D = np.zeros((nb * n, nb * n))
    for j in range(nb):
        D[j * n:(j + 1) * n, j * n:(j + 1) * n] = blocks[j]
    return D


# ---------------------------------------------------------------------------
# Schur complement Lambda_{kl} = sum_j tr(B_{k,j} Z_j^{-1} B_{l,j} X_j)
# (Alg. 2, eq. T2; Section IV-A, Omega).
# ---------------------------------------------------------------------------

def schur_dense(sdp: PolyaSDP, X: np.ndarray, Zi: np.ndarray) -> np.ndarray:
    """tr(B_k Z^{-1} B_l X) with every B_k materialised (tiny problems)."""
    Xd, Zd = blockdiag(X), blockdiag(Zi)
    Bs = [sdp.dense_B(k) for k in range(sdp.K)]
    out = np.empty((sdp.K, sdp.K))
    for k in range(sdp.K):
        left = Bs[k] @ Zd
        for l in range(sdp.K):
            out[k, l] = np.trace(left @ Bs[l] @ Xd)
    return out


def schur_definition(sdp: PolyaSDP, X: np.ndarray, Zi: np.ndarray) -> np.ndarray:
    """Column l of Omega is B(Z^{-1} B^T(e_l) X) (Section IV-A)."""
    return schur_definition_columns(sdp, X, Zi, range(sdp.K))


def schur_definition_columns(sdp: PolyaSDP, X: np.ndarray, Zi: np.ndarray, cols) -> np.ndarray:
    """The columns cols of Omega by the definition, [K][len(cols)]."""
    cols = list(cols)
    out = np.empty((sdp.K, len(cols)))
    e = np.zeros(sdp.K)
    for i, l in enumerate(cols):
        e[:] = 0.0
        e[l] = 1.0
        W = np.einsum("jab,jbc,jcd->jad", Zi, sdp.BT(e), X)
        out[:, i] = sdp.B(W)
    return out


def _sym_gather(F: np.ndarray, n: int) -> np.ndarray:
    """Sum F[(a,b),(c,d)] over (a,b) in S(p,q) and (c,d) in S(r,s) where
    S(p,q) = {(p,q),(q,p)} for p != q and {(p,p)} otherwise."""
    pairs = basis_pairs(n)
    p = np.array([x[0] for x in pairs])
    q = np.array([x[1] for x in pairs])
    i1 = p * n + q
    i2 = q * n + p
    w = (p != q).astype(np.float64)
    G = (F[np.ix_(i1, i1)] + w[:, None] * F[np.ix_(i2, i1)]
         + w[None, :] * F[np.ix_(i1, i2)] + (w[:, None] * w[None, :]) * F[np.ix_(i2, i2)])
    return G


def schur_expanded(sdp: PolyaSDP, X: np.ndarray, Zi: np.ndarray) -> np.ndarray:
    """Same matrix through the expansion of each block's trace into products
    of entries: with E = e_a e_b^T and E' = e_c e_d^T,
        tr(E Z^-1 E' X) = Zi[b,c] X[d,a]                                (P-block)
        tr((H^T E + E H) Zi (H'^T E' + E' H') X)
          = sum_t T_t[b,c] U_t[d,a],  (T,U) in {(Zi H'^T, X H^T), (Zi, H' X H^T),
                                            (H Zi H'^T, X), (H Zi, H' X)}.
    For a pair (h, h') the sum over blocks and terms is one product of the
    stacked, flattened T and U matrices."""
    n, Nt, L, L0 = sdp.n, sdp.Nt, sdp.L, sdp.L0
    out = np.zeros((sdp.K, sdp.K))
    for h in range(L0):
        for h2 in range(h, L0):
            Ts, Us = [], []
            for j in range(L):
                c = sdp.beta[h, j] * sdp.beta[h2, j]
                if c != 0.0:
                    Ts.append(c * Zi[j])
                    Us.append(X[j])
            for m in range(sdp.M):
                H1, H2 = sdp.H[m, h], sdp.H[m, h2]
                if not (np.any(H1) and np.any(H2)):
                    continue
                Zm, Xm = Zi[L + m], X[L + m]
                Ts += [Zm @ H2.T, Zm, H1 @ Zm @ H2.T, H1 @ Zm]
                Us += [Xm @ H1.T, H2 @ Xm @ H1.T, Xm, H2 @ Xm]
            if not Ts:
                continue
            T = np.stack(Ts).reshape(len(Ts), n * n)
            U = np.stack(Us).reshape(len(Us), n * n)
            R = T.T @ U                                   # R[(b,c),(d,a)]
            F = R.reshape(n, n, n, n).transpose(3, 0, 1, 2).reshape(n * n, n * n)
            blk = _sym_gather(F, n)
            out[h * Nt:(h + 1) * Nt, h2 * Nt:(h2 + 1) * Nt] = blk
            if h2 != h:
                out[h2 * Nt:(h2 + 1) * Nt, h * Nt:(h + 1) * Nt] = blk.T
    return out

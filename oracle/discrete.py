"""Discrete-time robust stability through the generalized LMI form (oracle).
Test infrastructure only.

The paper notes that the Lyapunov condition has a discrete-time counterpart
(Section II, after Theorem 1) and that the set-up extends to LMIs of the form
sum_i (A~_i X~ B~_i + B~_i^T X~ A~_i^T + R_i) < 0 (Section III-C, eq.
LMI_general), giving no formulas for either.  The reading used here (the
derivation is ours):

* x_{k+1} = A(alpha) x_k is stable for every alpha in the simplex iff there is
  P(alpha) > 0 with A^T P A - P < 0 there.  For P > 0 this is the 2n x 2n LMI
      M(alpha) = [[P, P A], [A^T P, P]] > 0
  (its Schur complement with respect to the leading P is P - A^T P A), and
  -M is eq. LMI_general with X~ = P, A~_1 = [I; 0], B~_1 = [-I/2, -A],
  A~_2 = [0; I], B~_2 = [0, -I/2], R = 0.
* With A homogeneous of degree da and P of degree dp, the diagonal blocks are
  made homogeneous of degree dp + da by (sum alpha)^da; Polya's multiplier
  (sum alpha)^d2 then gives, for every gamma in W_{dp+da+d2}, the coefficient
      M_gamma = sum_h [[b_{h,gamma} P_h, P_h H_{h,gamma}],
                       [H_{h,gamma}^T P_h, b_{h,gamma} P_h]],
  b_{h,gamma} = (da+d2)! / (gamma-h)!  (the coefficient of alpha^gamma in
  alpha^h (sum alpha)^{da+d2}; 0 unless gamma >= h) and H_{h,gamma} exactly
  as in the continuous set-up (eq. H_init / H with |lambda| = da).
* With Hh = [[-b/2 I, -H], [0, -b/2 I]] and Eh = blockdiag(E, E),
  M_gamma = -sum_h (Hh^T Eh_b + Eh_b Hh) y_(h,b): the derivative block of the
  continuous form at order 2n, with the basis matrices E_b replaced by
  blockdiag(E_b, E_b).  The P-blocks are kept at order 2n too
  (blockdiag(beta P, beta P), the same constraint twice) so that every block
  of the SDP has one order; C_j = delta s_j I (P-blocks) and eps s_j I
  (derivative blocks), the continuous form's reading of eq. C / Cj.

Everything else (the dual variable y of K = L0 n(n+1)/2 entries, the
objective a = 1, the IPM, phase-I and the certificate check) is the
continuous form's.  The Schur complement is taken by its definition
(columns B(Z^-1 B^T(e_l) X)).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import polya
from .sdp import PolyaSDP, basis_matrix, inner_basis, schur_definition, vec_to_sym


def _b_coef(l: int, dp: int, da: int, d2: int) -> np.ndarray:
    """b[h][m] = coefficient of alpha^{gamma_m} in alpha^h (sum alpha)^{da+d2}."""
    Wp = polya.monomials(l, dp)
    WM = polya.monomials(l, dp + da + d2)
    out = np.zeros((len(Wp), len(WM)))
    for hi, h in enumerate(Wp):
        for mi, g in enumerate(WM):
            diff = [gi - hj for gi, hj in zip(g, h)]
            if min(diff) >= 0:
                out[hi, mi] = polya.multinomial(da + d2, diff)
    return out


@dataclass
class DiscretePolyaSDP(PolyaSDP):
    """The SDP above for x+ = A(alpha) x; n is the system order, every block
    has order 2n."""

    def build(self) -> "DiscretePolyaSDP":
        super().build()                    # L0, L, M, Nt, K, beta, H, scales
        n = self.n
        self.bcoef = _b_coef(self.l, self.dp, self.da, self.d2)   # [L0][M]
        I = np.eye(n)
        self.Hh = np.zeros((self.M, self.L0, 2 * n, 2 * n))
        for m in range(self.M):
            for h in range(self.L0):
                b = self.bcoef[h, m]
                self.Hh[m, h, :n, :n] = -0.5 * b * I
                self.Hh[m, h, n:, n:] = -0.5 * b * I
                self.Hh[m, h, :n, n:] = -self.H[m, h]
        return self

    @property
    def bn(self) -> int:
        return 2 * self.n

    @property
    def pn(self) -> int:
        return self.n

    @property
    def m(self) -> int:
        return self.nb * self.bn

    def C_blocks(self) -> np.ndarray:
        return self.cdiag[:, None, None] * np.eye(self.bn)[None]

    def _hat(self, P: np.ndarray) -> np.ndarray:
        n = self.n
        out = np.zeros((2 * n, 2 * n))
        out[:n, :n] = P
        out[n:, n:] = P
        return out

    def BT(self, y: np.ndarray) -> np.ndarray:
        P = self.P_of_y(y)
        Ph = [self._hat(P[h]) for h in range(self.L0)]
        out = np.zeros((self.nb, self.bn, self.bn))
        for j in range(self.L):
            for h in range(self.L0):
                if self.beta[h, j] != 0.0:
                    out[j] += self.beta[h, j] * Ph[h]
        for m in range(self.M):
            acc = np.zeros((self.bn, self.bn))
            for h in range(self.L0):
                Hm = self.Hh[m, h]
                acc += Hm.T @ Ph[h] + Ph[h] @ Hm
            out[self.L + m] = -acc
        return out

    def B(self, W: np.ndarray) -> np.ndarray:
        """B(W)_(h,b) = sum_j tr(B_(h,b),j W_j) with tr(Eh_b S) the sum of
        tr(E_b .) over the two diagonal n x n blocks of S."""
        n = self.n
        out = np.zeros(self.K)
        for h in range(self.L0):
            S = np.zeros((self.bn, self.bn))
            for j in range(self.L):
                if self.beta[h, j] != 0.0:
                    S += self.beta[h, j] * W[j]
            for m in range(self.M):
                Hm = self.Hh[m, h]
                Wm = W[self.L + m]
                S -= Wm @ Hm.T + Hm @ Wm
            out[h * self.Nt:(h + 1) * self.Nt] = inner_basis(S[:n, :n], n) + inner_basis(S[n:, n:], n)
        return out

    def dense_B(self, k: int) -> np.ndarray:
        h, b = divmod(k, self.Nt)
        Eh = self._hat(basis_matrix(self.n, b))
        bn = self.bn
        D = np.zeros((self.m, self.m))
        for j in range(self.L):
            D[j * bn:(j + 1) * bn, j * bn:(j + 1) * bn] = self.beta[h, j] * Eh
        for m in range(self.M):
            Hm = self.Hh[m, h]
            jj = self.L + m
            D[jj * bn:(jj + 1) * bn, jj * bn:(jj + 1) * bn] = -(Hm.T @ Eh + Eh @ Hm)
        return D

    def dense_C(self) -> np.ndarray:
        return np.diag(np.repeat(self.cdiag, self.bn))

    def schur(self, X: np.ndarray, Zi: np.ndarray) -> np.ndarray:
        return schur_definition(self, X, Zi)

    def M_of_y(self, y: np.ndarray) -> np.ndarray:
        """The derivative blocks of B^T(y): the Polya coefficients M_gamma."""
        return self.BT(y)[self.L:]


def make_discrete_sdp(A: np.ndarray, n: int, l: int, dp: int, d: int, *, da: int = 1,
                      d1: int | None = None, d2: int | None = None, delta: float = 1e-3,
                      eps: float = 1e-3) -> DiscretePolyaSDP:
    return DiscretePolyaSDP(n=n, l=l, dp=dp, da=da, d1=d if d1 is None else d1,
                            d2=d if d2 is None else d2, A=np.asarray(A, dtype=np.float64),
                            delta=delta, eps=eps).build()


def lyapunov_margin(A_of: callable, P_of: callable, alphas) -> tuple:
    """Brute-force check of a certificate at simplex points: the smallest
    eigenvalue of P(alpha) and the largest of A^T P A - P."""
    lo, hi = np.inf, -np.inf
    for a in alphas:
        Aa, Pa = A_of(a), P_of(a)
        lo = min(lo, float(np.linalg.eigvalsh(Pa)[0]))
        hi = max(hi, float(np.linalg.eigvalsh(Aa.T @ Pa @ Aa - Pa)[-1]))
    return lo, hi

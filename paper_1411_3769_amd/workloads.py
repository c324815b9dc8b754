"""Seeded synthetic workloads (uncertain affine systems on the simplex).

This module only draws random vertex matrices; it holds none of the method's
arithmetic.  It is the one piece shared by the FP64 oracle and the GPU path:
both receive the same host arrays.

The paper's numerical examples use "random" systems (Example 3) and a tokamak
model whose vertex matrices are not printed (Example 1), so every workload here
is synthetic.  Draw order is fixed and documented per family so that a seed
always maps to the same matrices.

Families (sizes follow the configurations the solver is measured on):

* ``plain``   n=4, l=3, dp=d=1.  G_1..G_l ~ N(0,1)^{n x n} drawn in order;
              A_i = G_i - (max Re eig(G_i) + 1) I.  The infeasible twin shifts
              A_1 by +2I (its vertex then has max Re eig = +1).
* ``dissip``  A_0 = -(S S^T / n + 0.5 I) + (Kmat - Kmat^T),
              A_i = A_0 + s * E_i / sqrt(n); draws S, Kmat, E_1..E_l in order.
              Used at (n=10, l=4, dp=d=2), (n=100, l=4, dp=1, d=3) and the
              warm-start family (n=32, l=4, dp=1, d=2, s ~ U[0.1, 0.5] drawn
              first from the same stream).
* ``mixed``   a meta stream (seed 0) draws, per system, n ~ U{6..48},
              l ~ U{2..5}, dp ~ U{1,2}, d ~ U{1..4}, s ~ U[0.1, 0.5] and a
              64-bit child seed; vertices then come from ``dissip``.
* ``contract`` (discrete time, x+ = A(alpha) x) rho ~ U[0.6, 0.98] first,
              then G_1..G_l ~ N(0,1)^{n x n} in order; A_i = rho G_i / ||G_i||_2,
              so every A(alpha) on the simplex has norm <= rho.  Used at
              (n=8, l=4, dp=d=1), 64 seeds.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class System:
    """One uncertain system: vertices A[l][n][n] (row-major) and degrees."""

    A: np.ndarray
    n: int
    l: int
    dp: int
    d: int
    seed: int
    tag: str = ""
    form: str = "continuous"    # or "discrete": x+ = A(alpha) x


def plain_vertices(seed: int, n: int = 4, l: int = 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    out = np.empty((l, n, n))
    for i in range(l):
        G = rng.standard_normal((n, n))
        shift = np.max(np.linalg.eigvals(G).real) + 1.0
        out[i] = G - shift * np.eye(n)
    return out


def plain_twin(A: np.ndarray) -> np.ndarray:
    B = A.copy()
    B[0] = B[0] + 2.0 * np.eye(A.shape[1])
    return B


def dissip_vertices(seed: int, n: int, l: int, s: float = 0.3,
                    rng: np.random.Generator | None = None) -> np.ndarray:
    rng = np.random.default_rng(seed) if rng is None else rng
    S = rng.standard_normal((n, n))
    Km = rng.standard_normal((n, n))
    A0 = -(S @ S.T / n + 0.5 * np.eye(n)) + (Km - Km.T)
    out = np.empty((l, n, n))
    for i in range(l):
        E = rng.standard_normal((n, n))
        out[i] = A0 + s * E / np.sqrt(n)
    return out


def plain_system(seed: int, twin: bool = False) -> System:
    A = plain_vertices(seed)
    if twin:
        A = plain_twin(A)
    return System(A, 4, 3, 1, 1, seed, "plain-twin" if twin else "plain")


def c1_system(seed: int) -> System:
    """n=10, l=4, dp=d=2, s=0.3 (64 seeds are 0..63)."""
    return System(dissip_vertices(seed, 10, 4, 0.3), 10, 4, 2, 2, seed, "n10")


def c2_system(seed: int) -> System:
    """n=100, l=4, dp=1, d=3, s=0.3 (seeds 0..3)."""
    return System(dissip_vertices(seed, 100, 4, 0.3), 100, 4, 1, 3, seed, "n100")


def warm_system(seed: int) -> System:
    """n=32, l=4, dp=1, d=2 with s ~ U[0.1, 0.5] drawn first from the stream."""
    rng = np.random.default_rng(seed)
    s = float(rng.uniform(0.1, 0.5))
    return System(dissip_vertices(seed, 32, 4, s, rng=rng), 32, 4, 1, 2, seed, "n32")


def contract_vertices(seed: int, n: int, l: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    rho = float(rng.uniform(0.6, 0.98))
    out = np.empty((l, n, n))
    for i in range(l):
        G = rng.standard_normal((n, n))
        out[i] = rho * G / np.linalg.norm(G, 2)
    return out


def discrete_system(seed: int) -> System:
    """Discrete time: n=8, l=4, dp=d=1, contractive vertices (64 seeds 0..63)."""
    return System(contract_vertices(seed, 8, 4), 8, 4, 1, 1, seed, "d8", "discrete")


def mixed_systems(count: int = 512, meta_seed: int = 0) -> list[System]:
    meta = np.random.default_rng(meta_seed)
    out = []
    for i in range(count):
        n = int(meta.integers(6, 49))
        l = int(meta.integers(2, 6))
        dp = int(meta.integers(1, 3))
        d = int(meta.integers(1, 5))
        s = float(meta.uniform(0.1, 0.5))
        child = int(meta.integers(0, 2**63 - 1, dtype=np.int64))
        out.append(System(dissip_vertices(child, n, l, s), n, l, dp, d, child, f"mixed{i}"))
    return out


def paper_shape_system(n: int, l: int, seed: int = 0) -> System:
    """Shapes of the paper's speed-up runs: dp=1, d1=d2=1."""
    return System(dissip_vertices(seed, n, l, 0.3), n, l, 1, 1, seed, f"shape{n}x{l}")


def random_spd_blocks(seed: int, nblocks: int, n: int, cond: float = 10.0) -> np.ndarray:
    """Random symmetric positive definite blocks, used as fixed IPM iterates."""
    rng = np.random.default_rng(seed)
    out = np.empty((nblocks, n, n))
    for j in range(nblocks):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = np.exp(rng.uniform(0.0, np.log(cond), n))
        out[j] = (Q * ev) @ Q.T
        out[j] = 0.5 * (out[j] + out[j].T)
    return out


def mlp_init(dims, seed: int) -> np.ndarray:
    """Initial weights of the warm-start network, flattened as
    [W1, b1, W2, b2, ...] (W_i [dims[i+1] x dims[i]] row-major): W ~
    N(0, 1/fan_in), b = 0, drawn in FP32."""
    rng = np.random.default_rng(seed)
    parts = []
    for din, dout in zip(dims[:-1], dims[1:]):
        parts.append((rng.standard_normal((dout, din)) / np.sqrt(din)).astype(np.float32).ravel())
        parts.append(np.zeros(dout, np.float32))
    return np.concatenate(parts)

"""Learned warm start: data, training and use of the warm-start network.

A network maps the vertex matrices of an uncertain system (l n^2 inputs) to
an interior-point starting point for its SDP: the dual vector y (K values, in
the library's dual order) and the log block scales s_j of X (L+M values).
Labels come from cold solves on the GPU: the iterate at the first iteration
whose relative gap reaches ``label_gap`` (psdp_opts.label_gap).  The library
projects the prediction into the interior and falls back to a cold solve
whenever the warm run does not end certified, so a poor prediction costs time,
never a verdict.

Everything numerical runs in libpolyaipm (IPM, network forward / backward /
Adam); this module only batches, normalises and shuffles on the host.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np

from . import polyaipm as P
from . import workloads as W

LABEL_GAP = 1e-1


def features(systems: Sequence[W.System]) -> np.ndarray:
    """Flattened vertices, [count x l n^2] float32."""
    return np.stack([np.asarray(s.A, dtype=np.float64).ravel() for s in systems]).astype(np.float32)


@dataclass
class LabelSet:
    x: np.ndarray                      # [N x l n^2] float32
    y: np.ndarray                      # [N x (K + L + M)] float64: label y, label logx
    cold_iters: np.ndarray             # cold-start iterations
    cold_verdict: np.ndarray
    cold_seconds: float                # summed wall time of the cold batched solves
    reached: np.ndarray                # label iterate recorded


def solve_cold(systems: Sequence[W.System], batch: int = 256, label_gap: float = LABEL_GAP,
               log: Optional[Callable[[str], None]] = None, **opts) -> LabelSet:
    xs, ys, its, ver, ok = [], [], [], [], []
    secs = 0.0
    for b0 in range(0, len(systems), batch):
        part = systems[b0:b0 + batch]
        gs = P.polya_setup_batched([(s.A, s.n, s.l, s.dp, s.d) for s in part])
        t0 = time.perf_counter()
        rs = P.ipm_solve_batched(gs, label_gap=label_gap, **opts)
        secs += time.perf_counter() - t0
        for g, r in zip(gs, rs):
            hit = r.label_iter >= 0
            ok.append(hit)
            ys.append(np.concatenate([r.label_y, r.label_logx]) if hit
                      else np.concatenate([r.y, r.logx]))
            its.append(r.iterations + r.phase1_iterations)
            ver.append(r.verdict)
            g.close()
        xs.append(features(part))
        if log:
            log(f"cold solves {min(b0 + batch, len(systems))}/{len(systems)} ({secs:.1f} s)")
    return LabelSet(np.concatenate(xs), np.stack(ys), np.array(its), np.array(ver), secs,
                    np.array(ok))


@dataclass
class Normaliser:
    mean: np.ndarray
    std: np.ndarray

    @classmethod
    def fit(cls, v: np.ndarray) -> "Normaliser":
        mean = v.mean(axis=0)
        std = v.std(axis=0)
        std = np.maximum(std, 1e-6 * np.maximum(np.abs(mean), 1e-12) + 1e-30)
        return cls(mean, std)

    def fwd(self, v):
        return ((v - self.mean) / self.std).astype(np.float32)

    def inv(self, v):
        return np.asarray(v, dtype=np.float64) * self.std + self.mean


@dataclass
class WarmStartModel:
    dims: tuple
    net: P.MLP
    xnorm: Normaliser
    ynorm: Normaliser
    K: int
    history: List[float] = field(default_factory=list)

    def predict(self, x: np.ndarray, batch: int = 256):
        """Warm-start data (y list, logx list) for feature rows x."""
        import torch
        out = []
        for b0 in range(0, x.shape[0], batch):
            xb = torch.tensor(self.xnorm.fwd(x[b0:b0 + batch]), device="cuda")
            out.append(self.net.forward(xb).cpu().numpy())
        v = self.ynorm.inv(np.concatenate(out))
        return [row[:self.K] for row in v], [row[self.K:] for row in v]


def train(data: LabelSet, K: int, hidden=(1024, 1024), epochs: int = 60, batch: int = 256,
          lr: float = 1e-3, lr_final: float = 1e-4, seed: int = 0, precision: str = "bf16",
          log: Optional[Callable[[str], None]] = None) -> WarmStartModel:
    """Adam on the normalised MSE, learning rate decayed geometrically from lr
    to lr_final; the epoch order of samples comes from a seeded permutation."""
    import torch
    dims = (data.x.shape[1], hidden[0], hidden[1], data.y.shape[1])
    xn = Normaliser.fit(data.x.astype(np.float64))
    yn = Normaliser.fit(data.y)
    X = torch.tensor(xn.fwd(data.x), device="cuda")
    Y = torch.tensor(yn.fwd(data.y), device="cuda")
    net = P.MLP(dims, precision=precision, max_batch=batch)
    net.set_params(W.mlp_init(dims, seed))
    model = WarmStartModel(dims, net, xn, yn, K)
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    steps = max(1, epochs * (n // batch))
    decay = (lr_final / lr) ** (1.0 / steps)
    cur = lr
    for ep in range(epochs):
        perm = torch.tensor(rng.permutation(n), device="cuda")
        tot = 0.0
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            xb = X.index_select(0, idx).contiguous()
            yb = Y.index_select(0, idx).contiguous()
            tot += net.loss_grad(xb, yb)
            net.adam(lr=cur)
            cur *= decay
            nb += 1
        model.history.append(tot / max(nb, 1))
        if log and (ep % 10 == 0 or ep == epochs - 1):
            log(f"epoch {ep}: loss {model.history[-1]:.4e} lr {cur:.2e}")
    return model


def evaluate(model: WarmStartModel, systems: Sequence[W.System], cold: LabelSet, batch: int = 256,
             log: Optional[Callable[[str], None]] = None, **opts) -> dict:
    """Warm-started solves of the held-out systems against their cold solves:
    iterations, wall time (inference included) and the fallback rate."""
    import torch
    its, fb, used, agree = [], 0, 0, 0
    secs = 0.0
    for b0 in range(0, len(systems), batch):
        part = systems[b0:b0 + batch]
        gs = P.polya_setup_batched([(s.A, s.n, s.l, s.dp, s.d) for s in part])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wy, wl = model.predict(features(part))
        rs = P.ipm_solve_batched(gs, warm_y=wy, warm_logx=wl, **opts)
        secs += time.perf_counter() - t0
        for i, r in enumerate(rs):
            its.append(r.iterations + r.phase1_iterations + (r.warm_iterations if r.warm_fallback else 0))
            fb += int(r.warm_fallback)
            used += int(r.warm_used)
            agree += int(r.verdict == cold.cold_verdict[b0 + i])
        for g in gs:
            g.close()
        if log:
            log(f"warm solves {min(b0 + batch, len(systems))}/{len(systems)} ({secs:.1f} s)")
    return dict(systems=len(systems), warm_iters_mean=float(np.mean(its)),
                cold_iters_mean=float(np.mean(cold.cold_iters)), warm_seconds=secs,
                cold_seconds=cold.cold_seconds, fallback_rate=fb / len(systems),
                warm_used=used, verdicts_agree=agree)

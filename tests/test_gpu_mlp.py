"""Warm-start network kernels against the FP64 oracle network (marker: gpu).

FP32 products: forward output and every gradient within 1e-4 relative (in
max norm over each parameter block).  BF16 products: within 3e-2 (operands
rounded to 8 significant bits, FP32 accumulation).  Shapes are ragged with
respect to the 64 x 64 tiles and the depth-16 staging.
"""
import numpy as np
import pytest

from oracle import mlp
from paper_1411_3769_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    from paper_1411_3769_amd import polyaipm
    polyaipm.load()
    return polyaipm


def _data(dims, batch, seed):
    rng = np.random.default_rng(seed)
    flat = W.mlp_init(dims, seed)
    flat[:] += 0.05 * rng.standard_normal(flat.size).astype(np.float32)   # non-zero biases
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    t = rng.standard_normal((batch, dims[-1])).astype(np.float32)
    return flat, x, t


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 3e-2)])
@pytest.mark.parametrize("dims,batch", [((37, 70, 45, 29), 19), ((130, 64, 200, 3), 64)])
def test_forward_and_gradient(P, prec, tol, dims, batch):
    import torch
    flat, x, t = _data(dims, batch, 11)
    print(f"mlp {prec} {dims} batch={batch}", flush=True)
    net = P.MLP(dims, precision=prec, max_batch=batch)
    net.set_params(flat)
    xd = torch.tensor(x, device="cuda")
    td = torch.tensor(t, device="cuda")
    out = net.forward(xd).cpu().numpy()
    params = mlp.unflatten(flat.astype(np.float64), dims)
    want, _ = mlp.forward(params, x.astype(np.float64))
    assert _rel(out, want) <= tol
    loss = net.loss_grad(xd, td)
    wl, wg = mlp.loss_and_grad(params, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - wl) <= tol * wl
    g = mlp.unflatten(net.get_grad().astype(np.float64), dims)
    for (gW, gb), (wW, wb) in zip(g, wg):
        assert _rel(gW, wW) <= tol
        assert _rel(gb, wb) <= tol
    net.close()


def test_adam_step_matches_oracle(P):
    import torch
    dims, batch = (37, 70, 45, 29), 19
    flat, x, t = _data(dims, batch, 3)
    net = P.MLP(dims, precision="fp32", max_batch=batch)
    net.set_params(flat)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    params = mlp.unflatten(flat.astype(np.float64), dims)
    st = mlp.adam_init(params)
    for _ in range(3):
        net.loss_grad(xd, td)
        net.adam(lr=1e-3)
        _, g = mlp.loss_and_grad(params, x.astype(np.float64), t.astype(np.float64))
        params = mlp.adam_step(params, g, st, lr=1e-3)
    got = net.get_params().astype(np.float64)
    want = mlp.flatten(params)
    # Adam's early steps are about lr * sign(g): agree to a small part of lr
    assert np.max(np.abs(got - want)) <= 3e-5


def test_training_reduces_loss(P):
    import torch
    dims, batch = (32, 64, 64, 8), 128
    rng = np.random.default_rng(0)
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    M = rng.standard_normal((dims[0], dims[-1])).astype(np.float32) / np.sqrt(dims[0])
    t = np.tanh(x @ M).astype(np.float32)
    net = P.MLP(dims, precision="bf16", max_batch=batch)
    net.set_params(W.mlp_init(dims, 0))
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(t, device="cuda")
    l0 = net.loss_grad(xd, td)
    for _ in range(200):
        net.loss_grad(xd, td)
        net.adam(lr=3e-3)
    l1 = net.loss_grad(xd, td)
    assert l1 < 0.1 * l0


def test_full_size_forward_bf16(P):
    """4096 -> 1024 -> 1024 -> 2167 at batch 256 (the n=32 family's network):
    sampled rows against the oracle."""
    import torch
    dims, batch = (4096, 1024, 1024, 2167), 256
    flat = W.mlp_init(dims, 1)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((batch, dims[0])).astype(np.float32)
    net = P.MLP(dims, precision="bf16", max_batch=batch)
    net.set_params(flat)
    print("mlp full size", flush=True)
    out = net.forward(torch.tensor(x, device="cuda")).cpu().numpy()
    rows = [0, 77, 255]
    want, _ = mlp.forward(mlp.unflatten(flat.astype(np.float64), dims), x[rows].astype(np.float64))
    assert _rel(out[rows], want) <= 3e-2

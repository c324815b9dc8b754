"""Pins of the oracle's warm-start network (CPU): GELU special values and
its derivative against finite differences, the analytic gradient of the
loss against central finite differences, and Adam's first step."""
import numpy as np

from oracle import mlp
from paper_1411_3769_amd import workloads as W


def test_gelu_special_values():
    assert mlp.gelu(0.0) == 0.0
    assert abs(mlp.gelu(10.0) - 10.0) < 1e-20
    assert abs(mlp.gelu(-10.0)) < 1e-20
    assert mlp.gelu_grad(0.0) == 0.5
    # gelu(x) - gelu(-x) = x (Phi(x) + Phi(-x) = 1)
    x = np.linspace(-4, 4, 17)
    assert np.allclose(mlp.gelu(x) - mlp.gelu(-x), x, atol=1e-15)


def test_gelu_grad_finite_difference():
    x = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(fd, mlp.gelu_grad(x), atol=1e-9)


def _net(seed=0, dims=(7, 5, 6, 4)):
    flat = W.mlp_init(dims, seed).astype(np.float64)
    params = mlp.unflatten(flat, dims)
    rng = np.random.default_rng(seed + 1)
    # non-zero biases so that their gradient paths are exercised
    params = [(Wm, 0.1 * rng.standard_normal(b.shape)) for Wm, b in params]
    x = rng.standard_normal((3, dims[0]))
    t = rng.standard_normal((3, dims[-1]))
    return params, x, t, dims


def test_gradient_central_differences():
    params, x, t, dims = _net()
    loss, grads = mlp.loss_and_grad(params, x, t)
    flat = mlp.flatten(params)
    gflat = mlp.flatten(grads)
    h = 1e-6
    fd = np.empty_like(flat)
    for i in range(flat.size):
        e = np.zeros_like(flat)
        e[i] = h
        lp, _ = mlp.loss_and_grad(mlp.unflatten(flat + e, dims), x, t)
        lm, _ = mlp.loss_and_grad(mlp.unflatten(flat - e, dims), x, t)
        fd[i] = (lp - lm) / (2 * h)
    assert np.max(np.abs(fd - gflat)) <= 1e-8 * max(1.0, np.max(np.abs(gflat)))


def test_loss_definition():
    params, x, t, _ = _net(3)
    out, _ = mlp.forward(params, x)
    loss, _ = mlp.loss_and_grad(params, x, t)
    assert abs(loss - 0.5 * np.mean(np.sum((out - t) ** 2, axis=1))) <= 1e-15 * loss


def test_adam_first_step_moves_by_lr_times_sign():
    params, x, t, _ = _net(5)
    _, grads = mlp.loss_and_grad(params, x, t)
    st = mlp.adam_init(params)
    new = mlp.adam_step(params, grads, st, lr=1e-3, eps=0.0)
    for (W0, b0), (W1, b1), (gW, gb) in zip(params, new, grads):
        for p0, p1, g in ((W0, W1, gW), (b0, b1, gb)):
            nz = g != 0
            assert np.allclose((p0 - p1)[nz], 1e-3 * np.sign(g[nz]), rtol=1e-12)


def test_flatten_roundtrip():
    dims = (4, 3, 2)
    flat = W.mlp_init(dims, 2).astype(np.float64)
    assert np.array_equal(mlp.flatten(mlp.unflatten(flat, dims)), flat)
    assert flat.size == 4 * 3 + 3 + 3 * 2 + 2

"""Pins for the selector-network oracle: finite differences, torch autograd
(float64, CPU) and closed forms."""

import numpy as np
import pytest
import torch

from oracle import mlp as M

H, K = 16, 5


def data(B=37, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.normal(0, 0.4, M.param_count(H, K))
    X = rng.normal(0, 1, (B, M.NF))
    y = rng.integers(0, K, B)
    return p, X, y


def test_gradient_matches_central_differences():
    p, X, y = data()
    g = M.backward(p, X, y, H, K)
    h = 1e-6
    rng = np.random.default_rng(1)
    idx = rng.choice(p.size, 120, replace=False)
    num = np.empty(idx.size)
    for t, i in enumerate(idx):
        e = np.zeros_like(p)
        e[i] = h
        num[t] = (M.loss(p + e, X, y, H, K) - M.loss(p - e, X, y, H, K)) / (2 * h)
    assert np.max(np.abs(num - g[idx])) <= 1e-6 * max(1.0, np.max(np.abs(g[idx])))


def test_gradient_matches_torch_autograd():
    p, X, y = data(B=50, seed=3)
    W1, b1, W2, b2, W3, b3 = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in M.unpack(p, H, K)]
    Xt = torch.tensor(X)
    h1 = torch.relu(Xt @ W1.T + b1)
    h2 = torch.relu(h1 @ W2.T + b2)
    z = h2 @ W3.T + b3
    L = torch.nn.functional.cross_entropy(z, torch.tensor(y))
    L.backward()
    ref = np.concatenate([t.grad.numpy().ravel() for t in (W1, b1, W2, b2, W3, b3)])
    assert np.allclose(M.backward(p, X, y, H, K), ref, rtol=1e-10, atol=1e-12)
    assert M.loss(p, X, y, H, K) == pytest.approx(L.item(), rel=1e-12)
    _, _, _, prob = M.forward(p, X, H, K)
    assert np.allclose(prob, torch.softmax(z, 1).detach().numpy(), rtol=1e-12)


def test_zero_weights_closed_form():
    p = np.zeros(M.param_count(H, K))
    X = np.random.default_rng(2).normal(size=(9, M.NF))
    y = np.arange(9) % K
    _, _, _, prob = M.forward(p, X, H, K)
    assert np.allclose(prob, 1.0 / K)
    assert M.loss(p, X, y, H, K) == pytest.approx(np.log(K), abs=1e-15)
    g = M.backward(p, X, y, H, K)
    W1, b1, W2, b2, W3, b3 = M.unpack(g, H, K)
    # only the output bias receives gradient: mean(1/K - onehot)
    expect = np.full(K, 1.0 / K) - np.bincount(y, minlength=K) / 9.0
    assert np.allclose(b3, expect)
    assert not W1.any() and not W2.any() and not W3.any() and not b1.any() and not b2.any()


def test_adam_matches_torch():
    p, X, y = data(B=20, seed=5)
    g = M.backward(p, X, y, H, K)
    t = torch.tensor(p, requires_grad=True)
    opt = torch.optim.Adam([t], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    q = p.copy()
    for step in range(1, 4):
        t.grad = torch.tensor(g)
        opt.step()
        q, m, v = M.adam_step(q, g, m, v, step, lr=1e-2)
    assert np.allclose(q, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_decreases_loss():
    p, X, y = data(B=64, seed=7)
    y = (X[:, 0] > 0).astype(int) + 2 * (X[:, 1] > 0)    # a learnable rule, K >= 4
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    L0 = M.loss(p, X, y, H, K)
    for step in range(1, 301):
        p, m, v = M.adam_step(p, M.backward(p, X, y, H, K), m, v, step, lr=1e-2)
    assert M.loss(p, X, y, H, K) < 0.5 * L0

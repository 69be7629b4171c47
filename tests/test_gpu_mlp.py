"""The selector network's GPU kernels against the FP64 oracle."""

import numpy as np
import pytest

from oracle import mlp as M

pytestmark = pytest.mark.gpu

H, K = 64, 9


def batch(Bn=333, seed=0):
    rng = np.random.default_rng(seed)
    from paper_1003_0952_amd.selector import init_params
    p = init_params(H, K, seed).astype(np.float64) + rng.normal(0, 0.05, M.param_count(H, K))
    p[-K:] = rng.normal(0, 0.1, K)
    X = rng.normal(0, 1, (Bn, M.NF))
    y = rng.integers(0, K, Bn)
    return p.astype(np.float32), X.astype(np.float32), y.astype(np.int32)


def test_forward_backward_match_oracle():
    import torch
    from paper_1003_0952_amd.selector import GpuMlp
    p, X, y = batch()
    net = GpuMlp(torch, H, K, p)
    Xt = torch.from_numpy(X).cuda()
    yt = torch.from_numpy(y).cuda()
    act, logits, probs = net.forward(Xt)
    g = net.backward(Xt, yt, act, probs).cpu().numpy().astype(np.float64)
    p64, X64 = p.astype(np.float64), X.astype(np.float64)
    h1, h2, z, pr = M.forward(p64, X64, H, K)
    assert np.max(np.abs(logits.cpu().numpy() - z)) <= 1e-4 * max(1, np.abs(z).max())
    assert np.max(np.abs(probs.cpu().numpy() - pr)) <= 1e-5
    a = act.cpu().numpy().reshape(-1, 2 * H)
    assert np.max(np.abs(a[:, :H] - h1)) <= 1e-4 * max(1, np.abs(h1).max())
    ref = M.backward(p64, X64, y, H, K)
    assert np.linalg.norm(g - ref) <= 1e-4 * np.linalg.norm(ref)
    assert float(net.loss.cpu()[0]) == pytest.approx(M.loss(p64, X64, y, H, K), rel=1e-5)


def test_adam_matches_oracle_and_is_deterministic():
    import torch
    from paper_1003_0952_amd.selector import GpuMlp
    p, X, y = batch(Bn=200, seed=4)
    runs = []
    for _ in range(2):
        net = GpuMlp(torch, H, K, p)
        Xt, yt = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
        for _ in range(5):
            act, _, probs = net.forward(Xt)
            net.backward(Xt, yt, act, probs)
            net.adam(lr=1e-3)
        runs.append(net.params.cpu().numpy())
    assert np.array_equal(runs[0], runs[1])   # fixed-order sums: bit-identical
    q = p.astype(np.float64)
    m = np.zeros_like(q)
    v = np.zeros_like(q)
    for s in range(1, 6):
        q, m, v = M.adam_step(q, M.backward(q, X.astype(np.float64), y, H, K), m, v, s, lr=1e-3)
    assert np.max(np.abs(runs[0] - q)) <= 1e-5


def test_training_reduces_loss_and_host_predict_agrees():
    import torch
    from paper_1003_0952_amd import selector as S
    rng = np.random.default_rng(9)
    F = rng.normal(0, 1, (600, M.NF)).astype(np.float32)
    labels = ((F[:, 0] > 0).astype(int) + 2 * (F[:, 3] > 0.5) + 4 * (F[:, 7] < -0.5)).astype(np.int32)
    params, mean, scale, hist = S.train(torch, F, labels, K, steps=400, lr=3e-3, seed=1)
    assert hist[-1] < 0.3 * hist[0]
    model = S.Selector(params, mean, scale, H=H, candidates=[str(i) for i in range(K)])
    pred = np.array([model.predict(f) for f in F])
    acc = np.mean(pred == labels)
    assert acc > 0.9
    # host inference equals the oracle's arg-max on the standardised features
    _, _, _, pr = M.forward(params.astype(np.float64), (F - mean) / scale, H, K)
    assert np.mean(pr.argmax(1) == pred) > 0.99

"""FP64 oracle of the selector network -- TEST INFRASTRUCTURE.

A 12-H-H-K multilayer perceptron with ReLU hidden layers and a softmax
cross-entropy loss, written out from the definitions; parameters in one flat
vector laid out as W1[H,12] b1[H] W2[H,H] b2[H] W3[K,H] b3[K] (row-major,
W[out, in]).  The ReLU derivative at 0 is taken as 0.  Adam follows Kingma
and Ba (2015), Algorithm 1, with the bias corrections.

Pinned in tests/test_oracle_mlp.py by central finite differences, by torch's
autograd in float64 on the CPU, and by closed forms (zero weights give a
uniform softmax and a loss of ln K).
"""

import numpy as np

NF = 12


def param_count(H, K):
    return H * NF + H + H * H + H + K * H + K


def unpack(p, H, K):
    p = np.asarray(p, dtype=np.float64)
    o = 0
    W1 = p[o:o + H * NF].reshape(H, NF); o += H * NF
    b1 = p[o:o + H]; o += H
    W2 = p[o:o + H * H].reshape(H, H); o += H * H
    b2 = p[o:o + H]; o += H
    W3 = p[o:o + K * H].reshape(K, H); o += K * H
    b3 = p[o:o + K]; o += K
    assert o == p.size
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, W3.ravel(), b3])


def forward(p, X, H, K):
    """Hidden activations, logits and probabilities of a batch X[B, 12]."""
    W1, b1, W2, b2, W3, b3 = unpack(p, H, K)
    X = np.asarray(X, dtype=np.float64)
    h1 = np.maximum(X @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    z = h2 @ W3.T + b3
    e = np.exp(z - z.max(axis=1, keepdims=True))
    prob = e / e.sum(axis=1, keepdims=True)
    return h1, h2, z, prob


def loss(p, X, labels, H, K):
    """Mean cross-entropy -log softmax(z)[label]."""
    _, _, z, _ = forward(p, X, H, K)
    zmax = z.max(axis=1, keepdims=True)
    lse = zmax[:, 0] + np.log(np.exp(z - zmax).sum(axis=1))
    return float(np.mean(lse - z[np.arange(z.shape[0]), labels]))


def backward(p, X, labels, H, K):
    """Gradient of the mean cross-entropy by the chain rule, same layout as p."""
    W1, b1, W2, b2, W3, b3 = unpack(p, H, K)
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    h1, h2, z, prob = forward(p, X, H, K)
    d3 = prob.copy()
    d3[np.arange(B), labels] -= 1.0
    d3 /= B
    gW3 = d3.T @ h2
    gb3 = d3.sum(axis=0)
    d2 = (d3 @ W3) * (h2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(axis=0)
    d1 = (d2 @ W2) * (h1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gW3, gb3)


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (p, m, v).  step is 1-based."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

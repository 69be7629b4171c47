"""Learned variant selector: a 12-64-64-K perceptron over the structural
features of csrc_features, trained on the GPU by the library's own forward,
backward and Adam kernels on the autotuner's timings, used on the host by
csrc_mlp_predict_host.  Exhaustive tuning stays the fallback (no model file)
and the reference for regret.
"""

import ctypes
import json
import os

import numpy as np

from . import binding as B
from .binding import check, np_ptr, t_ptr, stream_ptr
from . import tuner

HIDDEN = 64
NF = B.NFEATURES
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_data", "model.json")


def param_count(H, K):
    return int(B.lib.csrc_mlp_param_count(H, K))


def init_params(H, K, seed):
    """He-uniform weights, zero biases (numpy, seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((NF, H), (H, H), (H, K)):
        lim = np.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class GpuMlp:
    """Device buffers and calls of the library's MLP kernels."""

    def __init__(self, torch, H, K, params):
        self.t = torch
        self.H, self.K = H, K
        self.P = param_count(H, K)
        self.params = torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda()
        self.m = torch.zeros(self.P, dtype=torch.float32, device="cuda")
        self.v = torch.zeros_like(self.m)
        self.grads = torch.zeros_like(self.m)
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        self.step = 0

    def forward(self, X):
        torch = self.t
        Bn = X.shape[0]
        act = torch.empty(Bn * 2 * self.H, dtype=torch.float32, device="cuda")
        logits = torch.empty(Bn * self.K, dtype=torch.float32, device="cuda")
        probs = torch.empty_like(logits)
        check(B.lib.csrc_mlp_forward(self.H, self.K, Bn, t_ptr(self.params), t_ptr(X), t_ptr(act),
                                     t_ptr(logits), t_ptr(probs), stream_ptr()), "csrc_mlp_forward")
        return act, logits.view(Bn, self.K), probs.view(Bn, self.K)

    def backward(self, X, labels, act, probs):
        torch = self.t
        Bn = X.shape[0]
        work = torch.empty(Bn * (2 * self.H + self.K), dtype=torch.float32, device="cuda")
        check(B.lib.csrc_mlp_backward(self.H, self.K, Bn, t_ptr(self.params), t_ptr(X), t_ptr(act),
                                      t_ptr(probs), t_ptr(labels), t_ptr(self.grads), t_ptr(self.loss),
                                      t_ptr(work), stream_ptr()), "csrc_mlp_backward")
        return self.grads

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        check(B.lib.csrc_mlp_adam(self.P, t_ptr(self.params), t_ptr(self.grads), t_ptr(self.m), t_ptr(self.v),
                                  self.step, lr, beta1, beta2, eps, stream_ptr()), "csrc_mlp_adam")


def standardise(F):
    mean = F.mean(axis=0)
    scale = F.std(axis=0)
    scale[scale == 0] = 1.0
    return mean.astype(np.float32), scale.astype(np.float32)


def train(torch, F, labels, K, H=HIDDEN, steps=2000, lr=3e-3, seed=0, batch=0):
    """Train on the GPU; returns (params, mean, scale, loss history)."""
    mean, scale = standardise(F)
    Xs = ((F - mean) / scale).astype(np.float32)
    X = torch.from_numpy(np.ascontiguousarray(Xs)).cuda()
    y = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.int32)).cuda()
    net = GpuMlp(torch, H, K, init_params(H, K, seed))
    rng = np.random.default_rng(seed + 1)
    hist = []
    n = X.shape[0]
    for s in range(steps):
        if batch and batch < n:
            idx = torch.from_numpy(np.sort(rng.choice(n, batch, replace=False))).cuda()
            Xb, yb = X[idx].contiguous(), y[idx].contiguous()
        else:
            Xb, yb = X, y
        act, _, probs = net.forward(Xb)
        net.backward(Xb, yb, act, probs)
        net.adam(lr=lr)
        if s % 50 == 0 or s == steps - 1:
            hist.append(float(net.loss.cpu()[0]))
    return net.params.cpu().numpy(), mean, scale, hist


class Selector:
    """A trained model: parameters, feature standardisation and candidates."""

    def __init__(self, params, mean, scale, H=HIDDEN, candidates=None):
        self.params = np.ascontiguousarray(params, dtype=np.float32)
        self.mean = np.ascontiguousarray(mean, dtype=np.float32)
        self.scale = np.ascontiguousarray(scale, dtype=np.float32)
        self.H = H
        self.candidates = candidates or [tuner.candidate_name(i) for i in range(len(tuner.CANDIDATES))]
        self.K = len(self.candidates)

    def predict(self, features):
        f = np.ascontiguousarray(features, dtype=np.float32)
        c = ctypes.c_int32(0)
        check(B.lib.csrc_mlp_predict_host(self.H, self.K, np_ptr(self.params), np_ptr(self.mean),
                                          np_ptr(self.scale), np_ptr(f), ctypes.byref(c)), "predict")
        return c.value

    def select(self, n, ia, ja, vdtype=B.F64):
        """Class for a matrix structure (host ia/ja) through csrc_select:
        the library computes the features and runs the network."""
        ia = np.ascontiguousarray(ia, dtype=np.int32)
        ja = np.ascontiguousarray(ja, dtype=np.int32)
        c = ctypes.c_int32(0)
        check(B.lib.csrc_select(n, np_ptr(ia), np_ptr(ja), vdtype, self.H, self.K, np_ptr(self.params),
                                np_ptr(self.mean), np_ptr(self.scale), ctypes.byref(c)), "csrc_select")
        return c.value

    def save(self, path=MODEL_PATH):
        with open(path, "w") as fh:
            json.dump({"hidden": self.H, "candidates": self.candidates, "params": self.params.tolist(),
                       "mean": self.mean.tolist(), "scale": self.scale.tolist()}, fh)

    @staticmethod
    def load(path=MODEL_PATH):
        if not os.path.exists(path):
            return None
        with open(path) as fh:
            d = json.load(fh)
        return Selector(np.array(d["params"]), np.array(d["mean"]), np.array(d["scale"]), d["hidden"],
                        d["candidates"])


def choose(A, torch=None, mats=None, xs=None, ys=None, model=None):
    """Candidate index for matrix A: the model's pick (the fixed choice if the
    library cannot plan that candidate for A), else exhaustive tuning."""
    from . import api as C
    model = model if model is not None else Selector.load()
    if model is not None:
        pick = model.predict(C.csrc_features(A.host_ia, A.host_ja, A.vdtype))
        for i in (pick, tuner.DEFAULT, tuner.FALLBACK, tuner.PLAIN):
            v, kw = tuner.CANDIDATES[i]
            try:
                C.Plan(A, v, **kw)
            except C.CsrcError:
                continue
            return i, "learned" if i == pick else "fixed"
    times, best = tuner.tune(torch, mats, xs, ys)
    return best, "tuned"

"""Batched products: many matrices of uneven size, 1..32 right-hand sides,
one persistent launch (and the same launch replayed as a HIP graph)."""

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W
from tests.helpers import oracle_csrc, rel_inf

pytestmark = pytest.mark.gpu


def make_batch(count, kind="uniform", n_hi=6000):
    out = []
    for m in range(count):
        a, X = W.batch_member(m, kind=kind, n_lo=200, n_hi=n_hi)
        out.append((a, X))
    return out


def setup(C, torch, batch, dtype):
    mats, Xs, Ys, refs = [], [], [], []
    for a, X in batch:
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, dtype)
        mats.append(A)
        Xs.append(torch.from_numpy(X).to("cuda", A.xdtype))
    return mats, Xs


BATCH_VARIANTS = ["owner", "private"]


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("transpose", [False, True])
def test_batched_matches_oracle(dtype, transpose, variant):
    import torch
    import paper_1003_0952_amd as C
    batch = make_batch(24)
    mats, Xs = setup(C, torch, batch, dtype)
    bp = C.BatchPlan(mats, [X.shape[1] for _, X in batch], ydtype="f64" if dtype == "f64" else "f32",
                     variant=variant)
    Ys = [torch.full((a.n, X.shape[1]), float("nan"), dtype=bp.ytorch, device="cuda") for a, X in batch]
    (C.csrc_spmv_t_batched if transpose else C.csrc_spmv_batched)(bp, Xs, Ys)
    torch.cuda.synchronize()
    for (a, X), Y in zip(batch, Ys):
        c = oracle_csrc(a)
        if dtype == "f64":
            ref = np.stack([(R.spmv_t if transpose else R.spmv)(c, np.ascontiguousarray(X[:, j]))
                            for j in range(X.shape[1])], axis=1)
            assert rel_inf(Y.cpu().numpy(), ref) <= 1e-12
        else:
            ov = {s: R.dequantize(c[s], "f32") for s in ("ad", "al", "au")}
            Xf = R.to_f32(X).astype(np.float64)
            got = Y.double().cpu().numpy()
            for j in range(X.shape[1]):
                xj = np.ascontiguousarray(Xf[:, j])
                f = R.spmv_t if transpose else R.spmv
                ref = f(c, xj, **ov)
                bound = R.accumulation_bound(c, xj, 2.0**-24, transpose, **ov) + 2.0**-24 * np.abs(ref)
                assert np.all(np.abs(got[:, j] - ref) <= bound)


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
def test_batched_integer_equals_single_products(variant):
    import torch
    import paper_1003_0952_amd as C
    batch = make_batch(16, kind="int")
    mats, Xs = setup(C, torch, batch, "f64")
    bp = C.BatchPlan(mats, [X.shape[1] for _, X in batch], variant=variant)
    Ys = [torch.empty((a.n, X.shape[1]), dtype=torch.float64, device="cuda") for a, X in batch]
    C.csrc_spmv_batched(bp, Xs, Ys)
    torch.cuda.synchronize()
    for (a, X), A, Xt, Y in zip(batch, mats, Xs, Ys):
        plan = C.Plan(A, variant, max_rhs=X.shape[1])
        Ysingle = torch.empty_like(Y)
        C.csrc_spmm(A, plan, Xt, Ysingle)
        torch.cuda.synchronize()
        assert torch.equal(Y, Ysingle)
        assert np.array_equal(Y.cpu().numpy(), R.spmm(oracle_csrc(a), X))


@pytest.mark.parametrize("variant", BATCH_VARIANTS)
def test_graph_replay_equals_direct_launch(variant):
    import torch
    import paper_1003_0952_amd as C
    batch = make_batch(20)
    mats, Xs = setup(C, torch, batch, "f64")
    bp = C.BatchPlan(mats, [X.shape[1] for _, X in batch], variant=variant)
    Ys = [torch.zeros((a.n, X.shape[1]), dtype=torch.float64, device="cuda") for a, X in batch]
    bp.bind(Xs, Ys)
    bp.run()
    torch.cuda.synchronize()
    direct = [Y.clone() for Y in Ys]
    g = bp.graph()
    for rep in range(4):
        for Y in Ys:
            Y.fill_(float("nan"))        # eager work between replays
        torch.cuda.synchronize()
        bp.launch_graph(g)
        torch.cuda.synchronize()
        for Y, D in zip(Ys, direct):
            assert rel_inf(Y.cpu().numpy(), D.cpu().numpy()) <= 1e-15, rep
    # transpose graph
    gt = bp.graph(transpose=True)
    bp.launch_graph(gt)
    torch.cuda.synchronize()
    for (a, X), Y in zip(batch, Ys):
        c = oracle_csrc(a)
        ref = np.stack([R.spmv_t(c, np.ascontiguousarray(X[:, j])) for j in range(X.shape[1])], axis=1)
        assert rel_inf(Y.cpu().numpy(), ref) <= 1e-12

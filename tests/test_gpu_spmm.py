"""GPU parity of multiple right-hand sides Y = A X and Y = A^T X (row-major
n x r blocks with a leading dimension), every variant, through the C ABI.
Each column must equal the oracle's product of that column."""

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W
from synth.values import block_vector
from tests.helpers import oracle_csrc, rel_inf

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "atomic", "private", "color", "owner"]


def run_mm(C, torch, host, X, variant, transpose, ld_pad=0, dtype="f64", **kw):
    A = C.Matrix(host, dtype)
    r = X.shape[1]
    plan = C.Plan(A, variant, max_rhs=max(r, 1), **kw)
    xd = A.xdtype
    Xt = torch.zeros((A.n, r + ld_pad), dtype=xd, device="cuda")
    Xt[:, :r] = torch.from_numpy(X).to("cuda", xd)
    Yt = torch.full((A.n, r + ld_pad), float("nan"), dtype=plan.ytorch, device="cuda")
    Xv, Yv = Xt[:, :r], Yt[:, :r]
    (C.csrc_spmm_t if transpose else C.csrc_spmm)(A, plan, Xv, Yv)
    torch.cuda.synchronize()
    Y = Yt.cpu().numpy().astype(np.float64)
    if ld_pad:
        assert np.all(np.isnan(Y[:, r:])), "padding columns were written"
    return Y[:, :r]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("r", [1, 2, 3, 5, 8, 13, 32])
def test_spmm_fp64(variant, r):
    import torch
    import paper_1003_0952_amd as C
    a, _ = W.hex_mesh(13)
    X = block_vector(a, r, 77)
    print(f"spmm hex13 variant {variant} r {r}", flush=True)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for transpose in (False, True):
        Y = run_mm(C, torch, host, X, variant, transpose, ld_pad=3)
        ref = (lambda XX: np.stack([(R.spmv_t if transpose else R.spmv)(c, np.ascontiguousarray(XX[:, j]))
                                    for j in range(r)], axis=1))(X)
        assert rel_inf(Y, ref) <= 1e-12, (variant, r, transpose)


@pytest.mark.parametrize("variant", VARIANTS)
def test_spmm_integer_bit_exact(variant):
    import torch
    import paper_1003_0952_amd as C
    a, _ = W.tet_mesh(5, kind="int")
    X = block_vector(a, 11, 5, kind="int")
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    Y = run_mm(C, torch, host, X, variant, False)
    assert np.array_equal(Y, R.spmm(c, X))


@pytest.mark.parametrize("variant", ["private", "owner"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_spmm_reduced_precision_columns(variant, dtype):
    """Reduced storage, r = 9 (a partial last column chunk): each column
    within the FP32 accumulation bound of the oracle on the stored values."""
    import torch
    import paper_1003_0952_amd as C
    a, _ = W.quad64()
    X = block_vector(a, 9, 3)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    Y = run_mm(C, torch, host, X, variant, False, dtype=dtype, ydtype="f32")
    ov = {s: R.dequantize(c[s], dtype) for s in ("ad", "al", "au")}
    Xf = R.to_f32(X).astype(np.float64)
    for j in range(9):
        xj = np.ascontiguousarray(Xf[:, j])
        ref = R.spmv(c, xj, **ov)
        bound = R.accumulation_bound(c, xj, 2.0**-24, **ov) + 2.0**-24 * np.abs(ref)
        assert np.all(np.abs(Y[:, j] - ref) <= bound)


def test_spmm_errors():
    import torch
    import paper_1003_0952_amd as C
    a, _ = W.quad64()
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    plan = C.Plan(A, "private", max_rhs=4)
    X = torch.zeros((A.n, 5), dtype=torch.float64, device="cuda")
    Y = torch.zeros((A.n, 5), dtype=torch.float64, device="cuda")
    with pytest.raises(C.CsrcError):       # r above the plan's max_rhs
        C.csrc_spmm(A, plan, X, Y)
    with pytest.raises(C.CsrcError) as e:  # overlapping blocks
        C.csrc_spmm(A, plan, X[:, :4], X[:, 1:5])
    assert e.value.status == -6

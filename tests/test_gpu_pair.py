"""y = A x and yt = A^T x together (csrc_spmv_pair): one pass over the
entries with a PRIVATE atomic-merge plan, the two products in sequence with
any other plan.  Bars as for the single products: FP64 <= 1e-12 relative
infinity norm against the oracle; FP32 values within the accumulation
bound on the stored values."""

import numpy as np
import pytest

from oracle import reference as R
from tests.helpers import small_cases, oracle_csrc, rel_inf
from tests.test_gpu_spmv import make_plan

pytestmark = pytest.mark.gpu

CASES = small_cases()
PLANS = ["private_atomic", "private", "plain", "color"]


def run_pair(torch, C, A, plan, x):
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
    yt = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
    C.csrc_spmv_pair(A, plan, xt, y, yt)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), yt.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("variant", PLANS)
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_pair_fp64(variant, case):
    import torch
    import paper_1003_0952_amd as C
    name, a, x = CASES[case]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    plan = make_plan(C, A, variant)
    y, yt = run_pair(torch, C, A, plan, x)
    c = oracle_csrc(a)
    assert rel_inf(y, R.spmv(c, x)) <= 1e-12, (name, variant)
    assert rel_inf(yt, R.spmv_t(c, x)) <= 1e-12, (name, variant)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_pair_reduced_precision(dtype):
    import torch
    import paper_1003_0952_amd as C
    name, a, x = CASES[[c[0] for c in CASES].index("tet7x3")]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, dtype)
    plan = C.Plan(A, "private", atomic_merge=1, ydtype="f32")
    y, yt = run_pair(torch, C, A, plan, x)
    c = oracle_csrc(a)
    ov = {s: R.dequantize(c[s], dtype) for s in ("ad", "al", "au")}
    xf = R.to_f32(x).astype(np.float64)
    for got, tr in ((y, False), (yt, True)):
        ref = (R.spmv_t if tr else R.spmv)(c, xf, **ov)
        bound = R.accumulation_bound(c, xf, 2.0**-24, tr, **ov) + 2.0**-24 * np.abs(ref)
        assert np.all(np.abs(got - ref) <= bound), (dtype, tr)


def test_pair_rejects_overlapping_outputs():
    import torch
    import paper_1003_0952_amd as C
    name, a, x = CASES[0]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    plan = C.Plan(A, "private", atomic_merge=1)
    xt = torch.from_numpy(x).cuda()
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(C.CsrcError) as e:
        C.csrc_spmv_pair(A, plan, xt, y, y)
    from paper_1003_0952_amd import binding as B
    assert e.value.status == B.ERR_ALIAS

"""Numerically symmetric storage (Sec. 2.2: au equals al and is stored once;
the descriptor's au is al), every variant, through the C ABI.

Bars: FP64 relative infinity-norm error <= 1e-12 against the FP64 oracle
for A x and A^T x; FP32 values within the accumulation bound of the oracle
on the stored values (as for two-array storage)."""

import numpy as np
import pytest

from oracle import reference as R
from tests.helpers import small_cases, oracle_csrc, rel_inf
from tests.test_gpu_spmv import make_plan

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "atomic", "private", "color", "owner", "private_atomic", "tile_color"]
CASES = small_cases("sym")


def run(torch, C, A, x, variant, transpose, **kw):
    plan = make_plan(C, A, variant, **kw)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
    (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_symmetric_storage_fp64(variant, case):
    import torch
    import paper_1003_0952_amd as C
    name, a, x = CASES[case]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64", symmetric=True)
    assert A.desc.au == A.desc.al
    c = oracle_csrc(a)
    ref = R.spmv(c, x)
    for tr in (False, True):
        y = run(torch, C, A, x, variant, tr)
        assert rel_inf(y, ref) <= 1e-12, (name, variant, tr)


@pytest.mark.parametrize("variant", ["private", "private_atomic"])
def test_symmetric_storage_fp32(variant):
    import torch
    import paper_1003_0952_amd as C
    name, a, x = CASES[[c[0] for c in CASES].index("tet7x3")]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f32", symmetric=True)
    c = oracle_csrc(a)
    ov = {s: R.dequantize(c[s], "f32") for s in ("ad", "al", "au")}
    xf = R.to_f32(x).astype(np.float64)
    ref = R.spmv(c, xf, **ov)
    bound = R.accumulation_bound(c, xf, 2.0**-24, False, **ov) + 2.0**-24 * np.abs(ref)
    for tr in (False, True):
        y = run(torch, C, A, x, variant, tr, ydtype="f32")
        assert np.all(np.abs(y - ref) <= bound), (variant, tr)


def test_symmetric_flag_checks_values():
    import paper_1003_0952_amd as C
    name, a, x = small_cases()[0]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    with pytest.raises(ValueError):
        C.Matrix(host, "f64", symmetric=True)

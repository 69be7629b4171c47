"""Rectangular matrices A = A_S + A_R (Sec. 2.1, Fig. 2b) through the C ABI:
y = A x (x has m entries) and y = A^T x (y has m entries), the square part
under several plans.  Bar: FP64 relative infinity-norm error <= 1e-12
against the oracle; integer-valued data bit-exact."""

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W
from tests.helpers import rel_inf
from tests.test_gpu_spmv import make_plan

pytestmark = pytest.mark.gpu

VARIANTS = ["private_atomic", "private", "plain", "color", "owner", "tile_color"]


def setup(C, side, kind, dtype="f64"):
    (n, m, rowptr, col, val), x = W.rect_mesh(side, kind=kind)
    (srp, scol, sval), r = C.csrc_rect_split(n, m, rowptr, col, val)
    host = C.csrc_from_csr(n, srp, scol, sval)
    A = C.Matrix(host, dtype)
    Rp = C.RectPart(r, dtype)
    c = R.csr_to_csrc(n, srp, scol, sval)
    return n, m, A, Rp, c, r, x


def run(torch, C, A, Rp, plan, x, transpose):
    n, m = A.n, Rp.m
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    y = torch.full((m if transpose else n,), float("nan"), dtype=plan.ytorch, device="cuda")
    (C.csrc_spmv_rect_t if transpose else C.csrc_spmv_rect)(A, Rp, plan, xt, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("side", [9, 17])
def test_rect_fp64(variant, side):
    import torch
    import paper_1003_0952_amd as C
    n, m, A, Rp, c, r, x = setup(C, side, "uniform")
    plan = make_plan(C, A, variant)
    y = run(torch, C, A, Rp, plan, x, False)
    assert rel_inf(y, R.spmv_rect(c, r, x)) <= 1e-12
    yt = run(torch, C, A, Rp, plan, x[:n], True)
    assert rel_inf(yt, R.spmv_rect_t(c, r, x[:n])) <= 1e-12


@pytest.mark.parametrize("variant", ["private_atomic", "private"])
def test_rect_integer_bit_exact(variant):
    import torch
    import paper_1003_0952_amd as C
    n, m, A, Rp, c, r, x = setup(C, 9, "int")
    plan = make_plan(C, A, variant)
    assert np.array_equal(run(torch, C, A, Rp, plan, x, False), R.spmv_rect(c, r, x))
    assert np.array_equal(run(torch, C, A, Rp, plan, x[:n], True), R.spmv_rect_t(c, r, x[:n]))


def test_rect_rejects_mismatched_part():
    import torch
    import paper_1003_0952_amd as C
    n, m, A, Rp, c, r, x = setup(C, 5, "uniform")
    Rf = C.RectPart(r, "f32")
    plan = C.Plan(A, "private")
    xt = torch.from_numpy(x).cuda()
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):         # the binding's check
        C.csrc_spmv_rect(A, Rf, plan, xt, y)
    import ctypes
    from paper_1003_0952_amd import binding as B
    st = B.lib.csrc_spmv_rect(ctypes.byref(A.desc), ctypes.byref(Rf.desc), plan.handle, B.t_ptr(xt),
                              B.t_ptr(y), B.t_ptr(plan.workspace), plan.ws_bytes, B.stream_ptr())
    assert st == B.ERR_ARG                  # and the library's own

"""GPU parity of y = A x and y = A^T x, every variant, FP64, through the C ABI.

Bar: relative infinity-norm error <= 1e-12 against the FP64 oracle;
integer-valued inputs bit-exact for every variant (all partial sums are
integers below 2^24, so every summation order is exact).
"""

import sys

import numpy as np
import pytest

from oracle import reference as R
from tests.helpers import small_cases, oracle_csrc, rel_inf

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "atomic", "private", "color", "owner", "private_atomic", "tile_color"]
TOL = 1e-12


def make_plan(C, A, variant, **kw):
    """Plan of a variant name; private_atomic is PRIVATE with the atomic merge."""
    if variant == "private_atomic":
        return C.Plan(A, "private", atomic_merge=1, **kw)
    return C.Plan(A, variant, **kw)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available()
    return torch


def run(torch, C, host, x, variant, transpose, dtype="f64", **kw):
    A = C.Matrix(host, dtype)
    plan = make_plan(C, A, variant, **kw)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
    (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64), plan


CASES = small_cases()
INT_CASES = small_cases("int")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_fp64_parity(torch_cuda, variant, case):
    import paper_1003_0952_amd as C
    name, a, x = CASES[case]
    print(f"case {name} variant {variant}", flush=True)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for transpose in (False, True):
        y, _ = run(torch_cuda, C, host, x, variant, transpose)
        ref = (R.spmv_t if transpose else R.spmv)(c, x)
        assert rel_inf(y, ref) <= TOL, (name, variant, transpose, rel_inf(y, ref))


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", range(len(INT_CASES)), ids=[c[0] for c in INT_CASES])
def test_integer_bit_exact(torch_cuda, variant, case):
    import paper_1003_0952_amd as C
    name, a, x = INT_CASES[case]
    print(f"case {name} variant {variant} (integer)", flush=True)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for transpose in (False, True):
        y, _ = run(torch_cuda, C, host, x, variant, transpose)
        ref = (R.spmv_t if transpose else R.spmv)(c, x)
        assert np.array_equal(y, ref), (name, variant, transpose)


@pytest.mark.parametrize("variant", ["atomic", "private", "owner", "color"])
@pytest.mark.parametrize("lanes", [2, 4, 8, 16, 32, 64])
def test_lane_widths(torch_cuda, variant, lanes):
    import paper_1003_0952_amd as C
    name, a, x = CASES[1]
    print(f"case {name} variant {variant} lanes {lanes}", flush=True)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for block in (64, 256, 512):
        y, _ = run(torch_cuda, C, host, x, variant, False, lanes=lanes, block=block, tile_work=1500)
        assert rel_inf(y, R.spmv(c, x)) <= TOL


def test_error_paths(torch_cuda):
    import paper_1003_0952_amd as C
    torch = torch_cuda
    name, a, x = CASES[0]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    plan = C.Plan(A, "private")
    xt = torch.from_numpy(x).cuda()
    with pytest.raises(C.CsrcError) as e:
        C.csrc_spmv(A, plan, xt, xt)
    assert e.value.status == -6
    other = C.Matrix(C.csrc_from_csr(*(lambda b: (b.n, b.rowptr, b.col, b.val))(CASES[2][1])), "f64")
    xo = torch.zeros(other.n, dtype=torch.float64, device="cuda")
    yo = torch.zeros(other.n, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):         # the binding's check
        C.csrc_spmv(other, plan, xo, yo)
    import ctypes
    from paper_1003_0952_amd import binding as B
    st = B.lib.csrc_spmv(ctypes.byref(other.desc), plan.handle, B.t_ptr(xo), B.t_ptr(yo),
                         B.t_ptr(plan.workspace), plan.ws_bytes, B.stream_ptr())
    assert st == -10                        # and the library's own (CSRC_ERR_PLAN)
    y = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    st = B.lib.csrc_spmv(ctypes.byref(A.desc), plan.handle, B.t_ptr(xt), B.t_ptr(y),
                         B.t_ptr(plan.workspace), 16, B.stream_ptr())
    assert st == -7


def test_empty_matrix(torch_cuda):
    import paper_1003_0952_amd as C
    host = C.csrc_from_csr(0, [0], [], [])
    A = C.Matrix(host, "f64")
    for v in VARIANTS:
        plan = make_plan(C, A, v)
        e = torch_cuda.zeros(0, dtype=torch_cuda.float64, device="cuda")
        C.csrc_spmv(A, plan, e, e)


def test_repeated_products_identical(torch_cuda):
    """Plans are immutable: products repeat (deterministic variants bit-identically)."""
    import paper_1003_0952_amd as C
    torch = torch_cuda
    name, a, x = CASES[1]
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    xt = torch.from_numpy(x).cuda()
    for v in VARIANTS:
        plan = make_plan(C, A, v)
        y1 = C.spmv(A, plan, xt).clone()
        y2 = C.spmv(A, plan, xt)
        torch.cuda.synchronize()
        assert rel_inf(y1.cpu().numpy(), y2.cpu().numpy()) <= 1e-15


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
@pytest.mark.parametrize("tile_work", [300, 1500, 6000])
def test_tile_colour_classes(torch_cuda, case, tile_work):
    """Bounded-stride colour classes of tiles: parity for small tiles (many
    tiles and classes); repeated products agree to rounding (the LDS
    additions inside a tile come in the order the waves run)."""
    import paper_1003_0952_amd as C
    torch = torch_cuda
    name, a, x = CASES[case]
    print(f"case {name} tile_color tile_work {tile_work}", flush=True)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for transpose in (False, True):
        y, plan = run(torch, C, host, x, "tile_color", transpose, tile_work=tile_work)
        ref = (R.spmv_t if transpose else R.spmv)(c, x)
        assert rel_inf(y, ref) <= TOL, (name, tile_work, transpose, rel_inf(y, ref))
        info = plan.info()
        assert 1 <= info["ncolors"] <= info["ntiles"]
        if name.startswith("hex17") and tile_work == 300:
            assert info["ncolors"] > 2, info
        y2, _ = run(torch, C, host, x, "tile_color", transpose, tile_work=tile_work)
        assert rel_inf(y, y2) <= 1e-15, (name, tile_work, transpose)


@pytest.mark.parametrize("tile_work", [300, 8192, 1 << 20])
def test_atomic_merge_repeated(torch_cuda, tile_work):
    """PRIVATE with the atomic merge clears y before adding into it.
    Repeated products on one workspace (A x, A^T x and the two-product
    call), y filled with NaN before each, stay bit-exact on integer data (a
    value left uncleared would stay NaN), and afterwards the workspace is
    byte-for-byte what the upload wrote (the product writes no plan state).
    Tile sizes give many tiles and a single tile."""
    import paper_1003_0952_amd as C
    from synth import workloads as W
    torch = torch_cuda
    cases = [c for c in INT_CASES if c[0] in ("hex17_natural", "banded7001", "powerlaw6000", "n1")]
    a40, x40 = W.hex_mesh(40, "natural", kind="int")
    cases.append(("hex40_natural", a40, x40))
    for name, a, x in cases:
        print(f"case {name} atomic merge repeated, tile_work {tile_work}", flush=True)
        c = oracle_csrc(a)
        ref, reft = R.spmv(c, x), R.spmv_t(c, x)
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, "f64")
        plan = C.Plan(A, "private", atomic_merge=1, tile_work=tile_work)
        before = plan.workspace.clone()
        xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
        y = torch.empty((A.n,), dtype=plan.ytorch, device="cuda")
        yt = torch.empty_like(y)
        for rep in range(6):
            y.fill_(float("nan"))
            yt.fill_(float("nan"))
            if rep % 3 == 2:
                C.csrc_spmv_pair(A, plan, xt, y, yt)
            else:
                C.csrc_spmv(A, plan, xt, y)
                C.csrc_spmv_t(A, plan, xt, yt)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy(), ref), (name, tile_work, rep)
            assert np.array_equal(yt.cpu().numpy(), reft), (name, tile_work, rep)
        assert torch.equal(plan.workspace, before), (name, tile_work)

"""csrc_spmv_noalloc (the product whose plan tables and partials live in the
library's static device array, for callers that cannot allocate) against
csrc_spmv with the same plan, through the C ABI: two calls in a row, the
second on a smaller matrix, each checked against the workspace product and
the oracle.  Collected last so that a failure cannot hide other tests."""

import ctypes

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(B, A, plan, x, y):
    return B.lib.csrc_spmv_noalloc(ctypes.byref(A.desc), plan.handle, B.t_ptr(x), B.t_ptr(y), B.stream_ptr())


# The merge pass keeps window sums in the partial buffer (part of the static
# array here); the atomic merge and the colour sweep use only the plan
# tables.  Inside a tile the LDS additions come in the order the waves run,
# so real-valued results agree to rounding (the FP64 bar, 1e-12 relative),
# and integer-valued ones (every order exact) bit for bit.
PLANS = [("private", {"tile_work": 2048}),
         ("private", {"tile_work": 2048, "atomic_merge": 1}),
         ("color", {})]


@pytest.mark.parametrize("kind", ["uniform", "int"])
@pytest.mark.parametrize("variant,kw", PLANS)
def test_noalloc_matches_workspace_product(variant, kw, kind):
    import torch
    import paper_1003_0952_amd as C
    from paper_1003_0952_amd import binding as B
    # a larger matrix first, then a smaller one: the second call must not
    # read anything the first left in the array
    for a, x in (W.hex_mesh(24, "natural", kind=kind), W.quad64(kind=kind)):
        print(f"noalloc {variant} {kw} {kind} n={a.n}", flush=True)
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, "f64")
        plan = C.Plan(A, variant, **kw)
        assert 0 < plan.ws_bytes <= B.NOALLOC_MAX_BYTES
        xt = torch.from_numpy(x).cuda()
        y_ws = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
        y_na = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
        C.csrc_spmv(A, plan, xt, y_ws)
        assert _noalloc(B, A, plan, xt, y_na) == B.OK
        torch.cuda.synchronize()
        got, want = y_na.cpu().numpy(), y_ws.cpu().numpy()
        ref = R.spmv(R.csr_to_csrc(a.n, a.rowptr, a.col, a.val), x)
        if kind == "int":
            assert np.array_equal(got, want) and np.array_equal(got, ref)
        else:
            assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_noalloc_repeated_calls():
    """Repeated calls agree (the array keeps the last call's contents;
    nothing depends on them): bit for bit on integer data, to rounding on
    real data."""
    import torch
    import paper_1003_0952_amd as C
    from paper_1003_0952_amd import binding as B
    for kind in ("int", "uniform"):
        a, x = W.hex_mesh(17, "random", kind=kind)
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, "f64")
        plan = C.Plan(A, "private", tile_work=1024)
        xt = torch.from_numpy(x).cuda()
        outs = []
        for _ in range(3):
            y = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
            assert _noalloc(B, A, plan, xt, y) == B.OK
            torch.cuda.synchronize()
            outs.append(y.cpu().numpy())
        for o in outs[1:]:
            if kind == "int":
                assert np.array_equal(o, outs[0])
            else:
                assert np.max(np.abs(o - outs[0])) <= 1e-12 * np.max(np.abs(outs[0]))


def test_noalloc_rejects_plan_beyond_the_array():
    """A plan needing more than CSRC_NOALLOC_MAX_BYTES is refused with
    CSRC_ERR_WORKSPACE before any device work (y is left untouched)."""
    import torch
    import paper_1003_0952_amd as C
    from paper_1003_0952_amd import binding as B
    from synth import patterns as P
    from synth.values import fill_values, vector
    a = P.banded(12000, 400, 1.0, 5)     # one-row tiles of 400 window slots: 38 MiB of partials
    fill_values(a, 1)
    x = vector(a, 2)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    A = C.Matrix(host, "f64")
    plan = C.Plan(A, "private", tile_work=1)
    assert plan.ws_bytes > B.NOALLOC_MAX_BYTES
    xt = torch.from_numpy(x).cuda()
    y = torch.full((A.n,), 7.0, dtype=torch.float64, device="cuda")
    assert _noalloc(B, A, plan, xt, y) == B.ERR_WORKSPACE
    torch.cuda.synchronize()
    assert bool(torch.all(y == 7.0))

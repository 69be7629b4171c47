"""Reduced-precision storage (FP32 / BF16 values, FP32 x, FP32 accumulation),
every variant, y in FP32 or FP64, with and without the compensated merge
(the atomic merge has no compensated form).

Bars (Higham's bound for sums of m rounded products in any order):
* against the FP64 oracle on the stored (dequantised) values and rounded x:
  |y_hat - y~| <= gamma_m(2^-24) (|A~| |x~|)_i            (accumulation only)
* against the FP64 oracle on the original FP64 data: the stated total bound
  (u_v + u_x + gamma_m(2^-24)(1+u_v)(1+u_x)) (|A| |x|)_i, u_v = 2^-24 or 2^-8
* integer-valued data: bit-exact (every sum is an integer below 2^24).
"""

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W
from tests.helpers import oracle_csrc, rel_inf

pytestmark = pytest.mark.gpu

VARIANTS = ["plain", "atomic", "private", "color", "owner", "private_atomic", "tile_color"]


def run(C, torch, host, x, variant, dtype, ydtype, transpose=False, **kw):
    A = C.Matrix(host, dtype)
    if variant == "private_atomic":
        plan = C.Plan(A, "private", ydtype=ydtype, atomic_merge=1, **kw)
    else:
        plan = C.Plan(A, variant, ydtype=ydtype, **kw)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", torch.float32)
    y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
    (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
@pytest.mark.parametrize("ydtype", ["f32", "f64"])
def test_reduced_precision_bounds(variant, dtype, ydtype):
    import torch
    import paper_1003_0952_amd as C
    a, x = W.tet_mesh(8)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    ov = {s: R.dequantize(c[s], dtype) for s in ("ad", "al", "au")}
    xf = R.to_f32(x).astype(np.float64)
    uv = R.UNIT_ROUNDOFF[dtype]
    m = R.row_terms(c)
    for transpose in (False, True):
        for comp in ((False,) if variant == "private_atomic" else (False, True)):
            y = run(C, torch, host, x, variant, dtype, ydtype, transpose, compensated=comp)
            f = R.spmv_t if transpose else R.spmv
            ref_stored = f(c, xf, **ov)
            acc_bound = R.accumulation_bound(c, xf, 2.0**-24, transpose, **ov)
            if ydtype == "f32":
                acc_bound = acc_bound + 2.0**-24 * np.abs(ref_stored)
            assert np.all(np.abs(y - ref_stored) <= acc_bound), (variant, dtype, transpose)
            ref64 = f(c, x)
            scale = R.abs_product(c, x, transpose)
            total = (uv + 2.0**-24 + R.gamma(m + 1, 2.0**-24) * (1 + uv) * (1 + 2.0**-24)) * scale
            assert np.all(np.abs(y - ref64) <= total)
            print(f"{variant} {dtype} y={ydtype} T={transpose} comp={comp}: rel_inf vs stored "
                  f"{rel_inf(y, ref_stored):.2e}, vs fp64 {rel_inf(y, ref64):.2e}")


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_reduced_precision_integer_exact(variant, dtype):
    import torch
    import paper_1003_0952_amd as C
    a, x = W.hex_mesh(11, "random", kind="int")
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for transpose in (False, True):
        y = run(C, torch, host, x, variant, dtype, "f32", transpose)
        assert np.array_equal(y, (R.spmv_t if transpose else R.spmv)(c, x))


def _rel_to_scale(y, ref, scale):
    return np.abs(y - ref) / np.maximum(scale, np.finfo(np.float64).tiny)


@pytest.mark.parametrize("transpose", [False, True])
def test_compensated_merge_recovers_accuracy(transpose):
    """Where the merge dominates the rounding, the compensated (TwoSum)
    merge wins accuracy back.  A banded matrix (half-bandwidth 384, full
    band, FP32 values, FP32 y) cut into one-row tiles: every row's own sum
    (dominated by the diagonal, ~385 |x_i|) then receives one FP32 window
    partial from each of the 384 rows above it.  Plain FP32 summation of
    those partials into the large running sum loses low-order bits at every
    step; TwoSum keeps them.  Both stay within the accumulation bound; the
    compensated error, measured against the FP64 oracle on the stored values
    row by row relative to (|A~||x~|)_i, is at least four times smaller in
    the largest row and in the root mean square."""
    import torch
    import paper_1003_0952_amd as C
    from synth import patterns as P
    from synth.values import fill_values, vector
    a = P.banded(4096, 384, 1.0, 11)
    fill_values(a, 12)
    x = vector(a, 13)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    ov = {s: R.dequantize(c[s], "f32") for s in ("ad", "al", "au")}
    xf = R.to_f32(x).astype(np.float64)
    f = R.spmv_t if transpose else R.spmv
    ref = f(c, xf, **ov)
    scale = R.abs_product(c, xf, transpose, **ov)
    bound = R.accumulation_bound(c, xf, 2.0**-24, transpose, **ov) + 2.0**-24 * np.abs(ref)
    A = C.Matrix(host, "f32")
    errs = {}
    for comp in (False, True):
        plan = C.Plan(A, "private", ydtype="f32", tile_work=1, compensated=comp)
        info = plan.info()
        assert info["ntiles"] == a.n and info["max_window"] == 384   # one row per tile
        xt = torch.from_numpy(x).to("cuda", torch.float32)
        y = torch.full((A.n,), float("nan"), dtype=torch.float32, device="cuda")
        (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
        torch.cuda.synchronize()
        yh = y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(yh - ref) <= bound), comp
        e = _rel_to_scale(yh, ref, scale)
        errs[comp] = (float(e.max()), float(np.sqrt(np.mean(e * e))))
    print(f"merge of 384 partials per row, FP32 y, transpose={transpose}: "
          f"plain max {errs[False][0]:.3e} rms {errs[False][1]:.3e}; "
          f"compensated max {errs[True][0]:.3e} rms {errs[True][1]:.3e}")
    assert errs[True][0] * 4 <= errs[False][0]
    assert errs[True][1] * 4 <= errs[False][1]


@pytest.mark.parametrize("transpose", [False, True])
def test_atomic_merge_fp64_output_recovers_accuracy(transpose):
    """The atomic merge adds every tile's window sums straight into y with
    hardware atomics, so it has no TwoSum form; its accurate form is an FP64
    y (FP32 or BF16 storage, ydtype f64): the merge then runs in FP64.  On
    the case of the compensated test (384 FP32 window partials per row) the
    FP64-output error against the FP64 oracle on the stored values is at
    least four times below the FP32-output error, in the largest row and in
    the root mean square, and both stay within the accumulation bound."""
    import torch
    import paper_1003_0952_amd as C
    from synth import patterns as P
    from synth.values import fill_values, vector
    a = P.banded(4096, 384, 1.0, 11)
    fill_values(a, 12)
    x = vector(a, 13)
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    ov = {s: R.dequantize(c[s], "f32") for s in ("ad", "al", "au")}
    xf = R.to_f32(x).astype(np.float64)
    f = R.spmv_t if transpose else R.spmv
    ref = f(c, xf, **ov)
    scale = R.abs_product(c, xf, transpose, **ov)
    bound = R.accumulation_bound(c, xf, 2.0**-24, transpose, **ov) + 2.0**-24 * np.abs(ref)
    A = C.Matrix(host, "f32")
    xt = torch.from_numpy(x).to("cuda", torch.float32)
    errs = {}
    for ydt in ("f32", "f64"):
        plan = C.Plan(A, "private", ydtype=ydt, tile_work=1, atomic_merge=1)
        assert plan.info()["ntiles"] == a.n
        y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
        (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
        torch.cuda.synchronize()
        yh = y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(yh - ref) <= bound), ydt
        e = _rel_to_scale(yh, ref, scale)
        errs[ydt] = (float(e.max()), float(np.sqrt(np.mean(e * e))))
    print(f"atomic merge of 384 partials per row, transpose={transpose}: "
          f"FP32 y max {errs['f32'][0]:.3e} rms {errs['f32'][1]:.3e}; "
          f"FP64 y max {errs['f64'][0]:.3e} rms {errs['f64'][1]:.3e}")
    assert errs["f64"][0] * 4 <= errs["f32"][0]
    assert errs["f64"][1] * 4 <= errs["f32"][1]


def _odd_tail_matrix(kind="int"):
    """A banded pattern on 2000 rows, then 7 rows with no stored entries below
    the diagonal, with an odd number of stored (lower) entries: the tile that
    holds the last entry reads an odd count from its even start, and the
    tiles of the trailing rows have no entries at all."""
    from synth import patterns as P
    from synth.values import fill_values, vector
    b = P.banded(2000, 5, 0.7, 21)
    rows = b.rows()
    lo = rows > b.col
    li, lj = rows[lo], b.col[lo].astype(np.int64)
    if len(li) % 2 == 0:
        li, lj = li[:-1], lj[:-1]
    a = P._from_lower_pairs(2007, li, lj, "banded_tail")
    fill_values(a, 22, kind)
    return a, vector(a, 23, kind)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_odd_tail_entry_is_counted_once(dtype):
    """The PRIVATE tile kernel reads value pairs, and a bfloat16 pair that
    straddles the end of the last tile's range would reach past the arrays;
    that tile streams all but its last entry and adds that entry's two
    products itself.  Integer data, bit-exact against the oracle, for one
    row per tile (trailing tiles with no entries), small and default tiles,
    both products and every way the tile sums reach y."""
    import torch
    import paper_1003_0952_amd as C
    a, x = _odd_tail_matrix()
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    k = len(host["ja"])
    assert k % 2 == 1 and host["ia"][a.n - 7] == k     # odd count; the last 7 rows store nothing
    ydt = "f64" if dtype == "f64" else "f32"
    A = C.Matrix(host, dtype)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    for tw in (1, 64, 1000, 0):
        for kw in ({"atomic_merge": 1}, {}, {"variant": "tile_color"}):
            kw = dict(kw)
            variant = kw.pop("variant", "private")
            plan = C.Plan(A, variant, tile_work=tw, ydtype=ydt, **kw)
            tiles = plan.export(0)
            last = int(np.searchsorted(tiles, a.n - 7, side="right")) - 1
            if tw == 1:
                assert tiles[-2] == a.n - 1 and last < len(tiles) - 2   # empty tiles at the end
            for transpose in (False, True):
                y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
                (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
                torch.cuda.synchronize()
                ref = (R.spmv_t if transpose else R.spmv)(c, x)
                got = y.cpu().numpy().astype(np.float64)
                assert np.array_equal(got, ref), (dtype, tw, variant, kw, transpose)


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_odd_tail_entry_every_variant(dtype):
    """The same odd-count matrix through the other tile kernels (atomic scatter,
    owner, row colours, plain) and through the fused pair product: their
    bfloat16 pair that straddles a tile's end takes its first value from a
    2-byte load.  Integer data, bit-exact."""
    import torch
    import paper_1003_0952_amd as C
    a, x = _odd_tail_matrix()
    c = oracle_csrc(a)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    ydt = "f64" if dtype == "f64" else "f32"
    A = C.Matrix(host, dtype)
    xt = torch.from_numpy(np.ascontiguousarray(x)).to("cuda", A.xdtype)
    ref = R.spmv(c, x)
    ref_t = R.spmv_t(c, x)
    for variant, kw in (("atomic", {"tile_work": 64}), ("atomic", {}), ("owner", {"tile_work": 64}),
                        ("owner", {}), ("color", {}), ("plain", {})):
        plan = C.Plan(A, variant, ydtype=ydt, **kw)
        for transpose, want in ((False, ref), (True, ref_t)):
            y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
            (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().astype(np.float64), want), (dtype, variant, kw, transpose)
    for tw in (1, 64, 0):
        plan = C.Plan(A, "private", tile_work=tw, ydtype=ydt, atomic_merge=1)
        y = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
        yt = torch.full((A.n,), float("nan"), dtype=plan.ytorch, device="cuda")
        C.csrc_spmv_pair(A, plan, xt, y, yt)
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().astype(np.float64), ref), (dtype, "pair", tw)
        assert np.array_equal(yt.cpu().numpy().astype(np.float64), ref_t), (dtype, "pair T", tw)

"""PRIVATE tiles whose windows have a chosen number of intervals.

The tile kernel is built for at most 2, 4 or 8 window intervals per tile
(the lookup compares against that many interval starts) and, beyond 8, falls
back to a search over the interval list in LDS.  Banded patterns with lower
neighbours at a few far-apart offsets give every tile one window interval
per offset, so each form runs: 2 intervals, 3 and 4, 7, and 11 (the LDS
search).  Integer values make every result exact: each form must reproduce
the oracle bit for bit, with the merge pass, the atomic merge, tile colour
classes and the two-product call.
"""

import ctypes

import numpy as np
import pytest

from oracle import reference as R
from synth import patterns as P
from synth.values import fill_values, vector
from tests.helpers import oracle_csrc

pytestmark = pytest.mark.gpu

N = 3000
TILE_WORK = 300
OFFSETS = {
    2: (1, 200),
    3: (1, 90, 180),
    4: (1, 60, 120, 180),
    7: (1, 60, 120, 180, 240, 300, 360),
    11: tuple(range(1, 600, 55)),
}


def offsets_matrix(n, offs, seed=5):
    """Lower neighbours of row i at i - d for every offset d (and the mirror
    entries above the diagonal), integer values."""
    i = np.arange(n, dtype=np.int64)
    li = np.concatenate([i[i >= d] for d in offs])
    lj = np.concatenate([i[i >= d] - d for d in offs])
    a = P._from_lower_pairs(n, li, lj, "offsets")
    fill_values(a, seed, "int")
    return a


def max_intervals(C, host):
    """Largest number of window intervals of one tile in the PRIVATE plan."""
    from paper_1003_0952_amd import binding as B
    opts = B.PlanOpts()
    B.check(B.lib.csrc_plan_opts_default(B.VARIANTS["private"], ctypes.byref(opts)))
    opts.tile_work = TILE_WORK
    h = ctypes.c_void_p(0)
    ia = np.ascontiguousarray(host["ia"], np.int32)
    ja = np.ascontiguousarray(host["ja"], np.int32)
    B.check(B.lib.csrc_plan_create(host["n"], B.np_ptr(ia), B.np_ptr(ja), 0, ctypes.byref(opts), ctypes.byref(h)))
    p = C.Plan.__new__(C.Plan)
    p._h = h
    iv = p.export(2).reshape(-1, 3)
    return int(np.bincount(iv[:, 0]).max())


@pytest.mark.parametrize("nint", sorted(OFFSETS))
def test_interval_counts_bit_exact(nint):
    import torch
    import paper_1003_0952_amd as C
    a = offsets_matrix(N, OFFSETS[nint])
    x = vector(a, 7, "int")
    c = oracle_csrc(a)
    ref, reft = R.spmv(c, x), R.spmv_t(c, x)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    assert max_intervals(C, host) == nint
    A = C.Matrix(host, "f64")
    xt = torch.from_numpy(x).to("cuda")
    for variant, kw in (("private", {}), ("private", {"atomic_merge": 1}), ("tile_color", {})):
        plan = C.Plan(A, variant, tile_work=TILE_WORK, **kw)
        for transpose, want in ((False, ref), (True, reft)):
            y = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
            (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
            torch.cuda.synchronize()
            print(f"{nint} intervals, {variant} {kw} T={transpose}", flush=True)
            assert np.array_equal(y.cpu().numpy(), want), (nint, variant, kw, transpose)
    plan = C.Plan(A, "private", tile_work=TILE_WORK, atomic_merge=1)
    y = torch.full((A.n,), float("nan"), dtype=torch.float64, device="cuda")
    yt = torch.full_like(y, float("nan"))
    C.csrc_spmv_pair(A, plan, xt, y, yt)
    torch.cuda.synchronize()
    assert np.array_equal(y.cpu().numpy(), ref) and np.array_equal(yt.cpu().numpy(), reft), nint


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_interval_counts_reduced_precision_exact(dtype):
    """The FP32 and BF16 kernels of every interval form, integer data (exact
    in both storage types)."""
    import torch
    import paper_1003_0952_amd as C
    for nint, offs in sorted(OFFSETS.items()):
        a = offsets_matrix(N, offs)
        x = vector(a, 7, "int")
        c = oracle_csrc(a)
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, dtype)
        xt = torch.from_numpy(x).to("cuda", torch.float32)
        plan = C.Plan(A, "private", tile_work=TILE_WORK, atomic_merge=1, ydtype="f32")
        for transpose, want in ((False, R.spmv(c, x)), (True, R.spmv_t(c, x))):
            y = torch.full((A.n,), float("nan"), dtype=torch.float32, device="cuda")
            (C.csrc_spmv_t if transpose else C.csrc_spmv)(A, plan, xt, y)
            torch.cuda.synchronize()
            assert np.array_equal(y.cpu().numpy().astype(np.float64), want), (dtype, nint, transpose)

"""The binding checks every tensor it passes to the library (type, length,
layout, device) and raises ValueError before any launch: the library takes
raw pointers and sizes, so a short or mistyped buffer would otherwise be read
or written past its end on the GPU.  Host-only: the checks run before the
library is called, with tensors in host memory."""

import numpy as np
import pytest
import torch

from paper_1003_0952_amd import api as C, binding as B
from synth import workloads as W


class FakePlan:
    """What the wrappers read from a plan before calling the library."""

    def __init__(self, n, vdtype, ydtype):
        self.n, self.vdtype, self.ydtype = n, vdtype, ydtype
        self.handle = None
        self.workspace = None
        self.ws_bytes = 0

    @property
    def ytorch(self):
        return torch.float64 if self.ydtype == B.F64 else torch.float32


@pytest.fixture(scope="module")
def mat():
    a, _ = W.quad64(side=8)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    return C.Matrix(host, "f64", device="cpu")


@pytest.fixture(scope="module")
def mat32():
    a, _ = W.quad64(side=8)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    return C.Matrix(host, "f32", device="cpu")


def vec(n, dt=torch.float64):
    return torch.zeros(n, dtype=dt)


@pytest.mark.parametrize("f", [C.csrc_spmv, C.csrc_spmv_t])
def test_vector_checks(mat, mat32, f):
    n = mat.n
    P = FakePlan(n, B.F64, B.F64)
    with pytest.raises(ValueError, match="dtype"):
        f(mat, P, vec(n, torch.float32), vec(n))            # x of the wrong type
    with pytest.raises(ValueError, match="dtype"):
        f(mat, P, vec(n), vec(n, torch.float32))            # y of the wrong type
    with pytest.raises(ValueError, match="elements"):
        f(mat, P, vec(n - 1), vec(n))                       # short x
    with pytest.raises(ValueError, match="elements"):
        f(mat, P, vec(n), vec(n - 1))                       # short y
    with pytest.raises(ValueError, match="contiguous"):
        f(mat, P, torch.zeros(2 * n, dtype=torch.float64)[::2], vec(n))
    with pytest.raises(ValueError, match="1-D"):
        f(mat, P, torch.zeros(n, 1, dtype=torch.float64), vec(n))
    with pytest.raises(TypeError):
        f(mat, P, np.zeros(n), vec(n))
    with pytest.raises(ValueError, match="another matrix"):
        f(mat, FakePlan(n + 1, B.F64, B.F64), vec(n), vec(n))
    with pytest.raises(ValueError, match="another matrix"):
        f(mat, FakePlan(n, B.F32_, B.F32_), vec(n), vec(n))
    # reduced storage: FP32 x; y as the plan says
    P32 = FakePlan(n, B.F32_, B.F32_)
    with pytest.raises(ValueError, match="dtype"):
        f(mat32, P32, vec(n), vec(n, torch.float32))
    with pytest.raises(ValueError, match="dtype"):
        f(mat32, P32, vec(n, torch.float32), vec(n))


def test_pair_checks(mat):
    n = mat.n
    P = FakePlan(n, B.F64, B.F64)
    with pytest.raises(ValueError, match="yt"):
        C.csrc_spmv_pair(mat, P, vec(n), vec(n), vec(n - 3))
    with pytest.raises(ValueError, match="dtype"):
        C.csrc_spmv_pair(mat, P, vec(n), vec(n), vec(n, torch.float32))


@pytest.mark.parametrize("f", [C.csrc_spmm, C.csrc_spmm_t])
def test_block_checks(mat, f):
    n = mat.n
    P = FakePlan(n, B.F64, B.F64)
    X = torch.zeros(n, 4, dtype=torch.float64)
    Y = torch.zeros(n, 4, dtype=torch.float64)
    with pytest.raises(ValueError, match="row-major"):
        f(mat, P, torch.zeros(4, n, dtype=torch.float64).t(), Y)   # a transposed view
    with pytest.raises(ValueError, match="columns"):
        f(mat, P, X, torch.zeros(n, 3, dtype=torch.float64))        # Y narrower than X
    with pytest.raises(ValueError, match="rows"):
        f(mat, P, X[: n - 1], Y)                                     # X short
    with pytest.raises(ValueError, match="dtype"):
        f(mat, P, X.float(), Y)
    with pytest.raises(ValueError, match="2-D"):
        f(mat, P, vec(n), Y)
    # a block with a row stride larger than r (a column slice of a wider block) is accepted by the checks
    wide = torch.zeros(n, 6, dtype=torch.float64)
    C._block(wide[:, :4], n, 4, torch.float64, "cpu", "X")


def test_rect_checks(mat):
    n = mat.n
    P = FakePlan(n, B.F64, B.F64)

    class R:
        pass
    r = R()
    r.n, r.m, r.vdtype = n, n + 5, B.F64
    with pytest.raises(ValueError, match="elements"):
        C.csrc_spmv_rect(mat, r, P, vec(n), vec(n))          # x needs m values
    with pytest.raises(ValueError, match="elements"):
        C.csrc_spmv_rect_t(mat, r, P, vec(n), vec(n))        # y needs m values
    r.vdtype = B.F32_
    with pytest.raises(ValueError, match="rectangular"):
        C.csrc_spmv_rect(mat, r, P, vec(n + 5), vec(n))

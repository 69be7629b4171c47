"""Pins for the oracle's product (Fig. 2a) and transpose (Sec. 5).

Each pin is independent of the oracle's own code: scipy's CSR product on the
original CSR matrix, numpy's dense product, exact integer arithmetic, closed
forms of special matrices, the adjoint identity and renumbering invariance.
A dropped term, a swapped al/au, a wrong index or sign fails at least one.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import reference as R
from synth import patterns as P, workloads as W
from synth.values import fill_values, vector


def rel_inf(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def scipy_A(a):
    return sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.n))


MATS = {
    "quad64": lambda: W.quad64(),
    "hex12": lambda: W.hex_mesh(12),
    "hex12_random": lambda: W.hex_mesh(12, "random"),
    "hex12_rcm": lambda: W.hex_mesh(12, "rcm"),
    "tet5x3": lambda: W.tet_mesh(5),
    "banded": lambda: (lambda a: (a, vector(a, 3)))(fill_values(P.banded(2000, 50, 0.2, 1), 2)),
    "power": lambda: (lambda a: (a, vector(a, 3)))(fill_values(P.power_law(3000, 20.0, 2.5, 5), 2)),
}


@pytest.mark.parametrize("name", list(MATS))
def test_product_matches_scipy_csr(name):
    a, x = MATS[name]()
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    A = scipy_A(a)
    y = R.spmv(c, x)
    assert rel_inf(y, A @ x) <= 1e-14
    yt = R.spmv_t(c, x)
    assert rel_inf(yt, A.T @ x) <= 1e-14
    # A is numerically non-symmetric: the two products differ
    assert rel_inf(y, yt) > 1e-3


def tiny_patterns():
    rng = np.random.default_rng(7)
    out = []
    n = 12
    # tridiagonal, arrow, full, empty rows, missing diagonals, random
    tri = np.zeros((n, n), bool)
    for i in range(n):
        tri[i, max(0, i - 1):i + 2] = True
    arrow = np.eye(n, dtype=bool)
    arrow[0, :] = arrow[:, 0] = True
    full = np.ones((n, n), bool)
    empty = np.zeros((n, n), bool)
    empty[3, 7] = empty[7, 3] = True
    nodiag = tri.copy()
    nodiag[np.arange(0, n, 2), np.arange(0, n, 2)] = False
    out += [tri, arrow, full, empty, nodiag]
    for m in (1, 2, 5, 31, 64):
        s = rng.random((m, m)) < 0.3
        s = s | s.T
        d = rng.random(m) < 0.7
        s[np.arange(m), np.arange(m)] = d
        out.append(s)
    return out


@pytest.mark.parametrize("idx", range(10))
def test_product_matches_dense(idx):
    pat = tiny_patterns()[idx]
    n = pat.shape[0]
    rng = np.random.default_rng(idx)
    D = np.where(pat, rng.uniform(-1, 1, (n, n)), 0.0)
    A = sp.csr_matrix(D)
    # keep explicit pattern even where the value happened to be 0
    rows, cols = np.nonzero(pat)
    vals = D[rows, cols]
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    c = R.csr_to_csrc(n, rowptr, cols, vals)
    x = rng.uniform(-1, 1, n)
    assert np.allclose(R.spmv(c, x), D @ x, rtol=1e-14, atol=1e-14)
    assert np.allclose(R.spmv_t(c, x), D.T @ x, rtol=1e-14, atol=1e-14)
    assert np.allclose(R.csrc_to_dense(c), D, rtol=0, atol=0)
    # the pure-Python loop follows the same order: bit-identical
    assert np.array_equal(R.spmv_py(c, x), R.spmv(c, x))
    assert np.array_equal(R.spmv_py(c, x, transpose=True), R.spmv_t(c, x))
    del A


def test_identity_and_diagonal_exact():
    n = 50
    c = R.csr_to_csrc(n, np.arange(n + 1), np.arange(n), np.ones(n))
    x = np.random.default_rng(1).uniform(-1, 1, n)
    assert np.array_equal(R.spmv(c, x), x)
    d = np.random.default_rng(2).uniform(-3, 3, n)
    c = R.csr_to_csrc(n, np.arange(n + 1), np.arange(n), d)
    assert np.array_equal(R.spmv(c, x), d * x)
    assert np.array_equal(R.spmv_t(c, x), d * x)


def test_laplacian_1d_exact():
    n = 100
    rows, cols, vals = [], [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i); cols.append(j); vals.append(2.0 if i == j else -1.0)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    c = R.csr_to_csrc(n, rowptr, np.array(cols), np.array(vals))
    y = R.spmv(c, np.ones(n))
    expect = np.zeros(n)
    expect[0] = expect[-1] = 1.0
    assert np.array_equal(y, expect)


def test_nine_point_laplacian_interior_zero():
    a = P.q1_quad(20, 20)
    rows = a.rows()
    a.val = np.where(rows == a.col, 8.0, -1.0)
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    y = R.spmv(c, np.ones(a.n))
    deg = np.diff(a.rowptr)
    assert np.array_equal(y, 8.0 - (deg - 1))
    assert np.all(y[deg == 9] == 0.0)


@pytest.mark.parametrize("name", ["quad64", "hex12_random", "tet5x3"])
def test_integer_values_exact(name):
    if name == "quad64":
        a, x = W.quad64(kind="int")
    elif name == "tet5x3":
        a, x = W.tet_mesh(5, kind="int")
    else:
        a, x = W.hex_mesh(12, "random", kind="int")
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    Ai = sp.csr_matrix((a.val.astype(np.int64), a.col, a.rowptr), shape=(a.n, a.n))
    xi = x.astype(np.int64)
    assert np.array_equal(R.spmv(c, x), (Ai @ xi).astype(np.float64))
    assert np.array_equal(R.spmv_t(c, x), (Ai.T @ xi).astype(np.float64))


def test_adjoint_identity():
    a, x = W.hex_mesh(10)
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    z = vector(a, 77)
    lhs = np.dot(x, R.spmv(c, z))
    rhs = np.dot(R.spmv_t(c, x), z)
    m = int(R.row_terms(c).max()) + 1
    scale = np.dot(np.abs(x), R.abs_product(c, z))
    assert abs(lhs - rhs) <= 2 * R.gamma(m + a.n, 2.0**-53) * scale


def test_renumbering_invariance():
    for ordering in ("random", "rcm"):
        a0, x0 = W.hex_mesh(9, kind="int")
        a1, x1 = W.hex_mesh(9, ordering, kind="int")
        c0 = R.csr_to_csrc(a0.n, a0.rowptr, a0.col, a0.val)
        c1 = R.csr_to_csrc(a1.n, a1.rowptr, a1.col, a1.val)
        # row r of the renumbered matrix is natural row orig[r]
        assert np.array_equal(x1, x0[a1.orig])
        assert np.array_equal(R.spmv(c1, x1), R.spmv(c0, x0)[a1.orig])
        assert np.array_equal(R.spmv_t(c1, x1), R.spmv_t(c0, x0)[a1.orig])


def test_spmm_columns_equal_spmv():
    a, _ = W.quad64()
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    from synth.values import block_vector
    X = block_vector(a, 5, 9)
    Y = R.spmm(c, X)
    for j in range(5):
        assert np.array_equal(Y[:, j], R.spmv(c, np.ascontiguousarray(X[:, j])))


def test_flop_and_load_model():
    # Sec. 4.1: CSRC takes n multiplies and nnz - n multiply-adds (2nnz - n
    # flops without FMA) and (5/2) nnz - n/2 loads: about 1.26 loads per flop
    # for the paper's matrices, against exactly 1.5 for CSR.
    n, nnz = 1_000_000, 26_463_592
    flops = 2 * nnz - n
    loads = 2.5 * nnz - 0.5 * n
    assert abs(loads / flops - 1.26) < 0.02
    assert 3 * nnz / (2 * nnz) == 1.5


@pytest.mark.parametrize("name", ["quad64", "hex12_random", "tet5x3"])
def test_numerically_symmetric_storage(name):
    """Sec. 2.2: for a numerically symmetric matrix the CSRC split gives
    au equal to al, A x equals A^T x, and both equal scipy's product."""
    make = {"quad64": lambda: W.quad64(kind="sym"), "hex12_random": lambda: W.hex_mesh(12, "random", kind="sym"),
            "tet5x3": lambda: W.tet_mesh(5, kind="sym")}[name]
    a, x = make()
    A = scipy_A(a)
    assert abs(A - A.T).max() == 0.0
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    assert np.array_equal(c["al"], c["au"])
    y = R.spmv(c, x)
    assert np.array_equal(y, R.spmv_t(c, x))
    assert rel_inf(y, A @ x) <= 1e-14


@pytest.mark.parametrize("side", [5, 9])
def test_rectangular_product(side):
    """Sec. 2.1 / Fig. 2b: A (n x m) = A_S + A_R.  The split rebuilds A
    exactly, and the oracle's A x and A^T x equal scipy's products with the
    whole rectangular matrix."""
    (n, m, rowptr, col, val), x = W.rect_mesh(side)
    A = sp.csr_matrix((val, col, rowptr), shape=(n, m))
    (srp, scol, sval), r = R.split_rect(n, m, rowptr, col, val)
    assert r["kr"] > 0 and np.all(r["jar"] >= n) and np.all(scol < n)
    S = sp.csr_matrix((sval, scol, srp), shape=(n, m))
    Rm = sp.csr_matrix((r["ar"], r["jar"], r["iar"]), shape=(n, m))
    assert abs(S + Rm - A).max() == 0.0
    c = R.csr_to_csrc(n, srp, scol, sval)
    assert rel_inf(R.spmv_rect(c, r, x), A @ x) <= 1e-14
    xt = x[:n]
    assert rel_inf(R.spmv_rect_t(c, r, xt), A.T @ xt) <= 1e-14

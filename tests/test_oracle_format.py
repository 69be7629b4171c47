"""Pins for the oracle's CSR -> CSRC split and for the input generators.

The split (Sec. 2) is checked bit-exactly against scipy's triangular split of
the same matrix; sizes against closed forms of the stencil patterns.
"""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import reference as R
from synth import patterns as P, workloads as W
from synth.values import fill_values


def scipy_csrc(a):
    """CSRC arrays built with scipy only: tril(A,-1) row-wise, triu(A,1)^T."""
    A = sp.csr_matrix((a.val, a.col, a.rowptr), shape=(a.n, a.n))
    L = sp.tril(A, -1, format="csr")
    L.sort_indices()
    U = sp.triu(A, 1, format="csr").T.tocsr()
    U.sort_indices()
    assert np.array_equal(L.indptr, U.indptr) and np.array_equal(L.indices, U.indices)
    return {"ia": L.indptr.astype(np.int32), "ja": L.indices.astype(np.int32),
            "al": L.data, "au": U.data, "ad": A.diagonal()}


CASES = [
    lambda: W.quad64()[0],
    lambda: W.hex_mesh(12)[0],
    lambda: W.hex_mesh(12, "random")[0],
    lambda: W.hex_mesh(12, "rcm")[0],
    lambda: W.tet_mesh(6)[0],
    lambda: fill_values(P.banded(3000, 37, 0.3, 5), 9),
    lambda: fill_values(P.reorder(P.power_law(5000, 12.0, 2.5, 3), P.random_order(5000, 4)), 8),
]


@pytest.mark.parametrize("make", CASES)
def test_split_matches_scipy_bit_exact(make):
    a = make()
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    s = scipy_csrc(a)
    for key in ("ia", "ja"):
        assert np.array_equal(c[key], s[key]), key
    for key in ("ad", "al", "au"):
        assert np.array_equal(c[key].view(np.uint64), s[key].view(np.uint64)), key
    assert c["k"] == (a.nnz - a.n) // 2


def test_unsorted_rows_give_the_same_split():
    a = W.hex_mesh(7)[0]
    rng = np.random.default_rng(0)
    col = a.col.copy()
    val = a.val.copy()
    for i in range(a.n):
        s, e = a.rowptr[i], a.rowptr[i + 1]
        p = rng.permutation(e - s) + s
        col[s:e] = a.col[p]
        val[s:e] = a.val[p]
    c1 = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    c2 = R.csr_to_csrc(a.n, a.rowptr, col, val)
    for key in c1:
        assert np.array_equal(np.asarray(c1[key]), np.asarray(c2[key]))


@pytest.mark.parametrize("nx,ny,nz", [(64, 64, 1), (5, 7, 1), (100, 100, 100), (3, 4, 5)])
def test_stencil_pattern_sizes_closed_form(nx, ny, nz):
    # 9-point: nnz = (3nx-2)(3ny-2); 27-point: prod (3n_d - 2)
    if nz == 1:
        a = P.q1_quad(nx, ny)
        nnz = (3 * nx - 2) * (3 * ny - 2)
    else:
        if nx * ny * nz > 1000 and nx == 100:
            nnz = 298 ** 3
            assert nnz == 26463592
            assert (nnz - 10**6) // 2 == 12731796
            return
        a = P.q1_hex(nx, ny, nz)
        nnz = (3 * nx - 2) * (3 * ny - 2) * (3 * nz - 2)
    assert a.nnz == nnz
    assert a.n == nx * ny * nz


def test_quad64_sizes():
    a, x = W.quad64()
    assert (a.n, a.nnz) == (4096, 36100)
    assert (a.nnz - a.n) // 2 == 16002


def test_kuhn_tet_sizes_closed_form():
    # 15-point node stencil (7 edge directions): edges along e_S for each
    # non-empty S; count of node pairs = prod over axes of (N - [axis in S]).
    N = 6
    edges = 0
    for s in range(1, 8):
        m = 1
        for ax in range(3):
            m *= N - ((s >> ax) & 1)
        edges += m
    a = P.kuhn_tet(N, N, N, 3)
    assert a.n == 3 * N ** 3
    assert a.nnz == 9 * (N ** 3 + 2 * edges)
    # full-size tetrahedral case: 80^3 nodes, 3 dofs
    N = 80
    e80 = sum(np.prod([N - ((s >> ax) & 1) for ax in range(3)]) for s in range(1, 8))
    assert 9 * (N ** 3 + 2 * e80) == 67746222
    assert (67746222 - 3 * N ** 3) // 2 == 33105111


def test_interior_row_lengths():
    a = P.q1_hex(5, 5, 5)
    lens = np.diff(a.rowptr)
    assert lens.max() == 27 and lens[2 + 5 * (2 + 5 * 2)] == 27
    t = P.kuhn_tet(5, 5, 5, 3)
    assert np.diff(t.rowptr).max() == 45


def test_missing_diagonal_gives_zero():
    # pattern: 3x3 with entries (0,1),(1,0),(2,2),(1,2),(2,1); rows 0,1 lack a_ii
    rowptr = np.array([0, 1, 3, 5])
    col = np.array([1, 0, 2, 1, 2])
    val = np.array([2.0, 3.0, 4.0, 5.0, 6.0])
    c = R.csr_to_csrc(3, rowptr, col, val)
    assert list(c["ad"]) == [0.0, 0.0, 6.0]
    assert list(c["ia"]) == [0, 0, 1, 2] and list(c["ja"]) == [0, 1]
    assert list(c["al"]) == [3.0, 5.0] and list(c["au"]) == [2.0, 4.0]


def test_error_paths():
    with pytest.raises(R.CsrcError):   # duplicate
        R.csr_to_csrc(2, [0, 2, 3], [0, 0, 1], [1.0, 1.0, 1.0])
    with pytest.raises(R.CsrcError):   # out of range
        R.csr_to_csrc(2, [0, 1, 2], [0, 2], [1.0, 1.0])
    with pytest.raises(R.CsrcError):   # not structurally symmetric
        R.csr_to_csrc(2, [0, 1, 3], [0, 0, 1], [1.0, 1.0, 1.0])
    c = R.csr_to_csrc(2, [0, 1, 3], [0, 0, 1], [1.0, 7.0, 1.0], pad=True)
    assert c["k"] == 1 and c["al"][0] == 7.0 and c["au"][0] == 0.0


def test_empty_and_diagonal_only():
    c = R.csr_to_csrc(0, [0], [], [])
    assert c["k"] == 0 and c["ia"].shape == (1,)
    c = R.csr_to_csrc(3, [0, 1, 2, 3], [0, 1, 2], [1.0, 2.0, 3.0])
    assert c["k"] == 0 and list(c["ad"]) == [1.0, 2.0, 3.0]


def test_paper_example_counts():
    # Sec. 2: the 9x9 example has 33 non-zeros; with a full diagonal the
    # number of stored pairs is k = (nnz - n) / 2 = 12, which is also the
    # number of direct conflicts quoted in Sec. 3.2.
    assert (33 - 9) // 2 == 12
    # Sec. 3.1: the example's three blocks hold 7, 5 and 21 non-zeros.
    assert 7 + 5 + 21 == 33

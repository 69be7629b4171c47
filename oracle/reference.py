"""CPU oracle (TEST INFRASTRUCTURE): CSRC format, product, transpose, setup.

Readings of the paper used here (each also listed in the design notes):

* 0-based indices; row i of the lower part spans ``ia[i] .. ia[i+1]-1``.
* ``ia``/``ja`` describe the strictly lower part row by row, columns ascending;
  ``al[k] = a[i, ja[k]]`` and ``au[k] = a[ja[k], i]`` (Sec. 2).
* ``k`` is the number of stored strictly-lower entries; a missing diagonal
  entry gives ``ad[i] = 0``.  A stored explicit zero counts as structural.
* The input must be structurally symmetric; duplicates and out-of-range
  columns are rejected.  ``pad=True`` symmetrises the pattern with zeros.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg use this.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class CsrcError(ValueError):
    pass


def lib():
    """The C oracle (plain sequential FP64), built with gcc if not yet built."""
    global _LIB
    if _LIB is None:
        from . import build as _b
        if not os.path.exists(_b.OUT):
            _b.build()
        L = ctypes.CDLL(_b.OUT)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        i64 = ctypes.c_int64
        L.oracle_csrc_spmv.argtypes = [i32, P, P, P, P, P, P, P]
        L.oracle_csrc_spmv.restype = None
        L.oracle_csrc_spmv_t.argtypes = [i32, P, P, P, P, P, P, P]
        L.oracle_csrc_spmv_t.restype = None
        L.oracle_csrc_spmm.argtypes = [i32, P, P, P, P, P, i32, P, i64, P, i64]
        L.oracle_csrc_spmm.restype = None
        L.oracle_csrc_color.argtypes = [i32, P, P, i32, P]
        L.oracle_csrc_color.restype = i32
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Format (Sec. 2)
# --------------------------------------------------------------------------

def csr_to_csrc(n, rowptr, col, val, pad=False):
    """Split a structurally symmetric CSR matrix into CSRC arrays (Sec. 2).

    Returns ``dict(n, k, ia, ja, ad, al, au)``: ``ia``/``ja`` int32, values
    float64.  Pinned bit-exact against scipy's ``tril``/``triu`` split.
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    if rowptr.shape != (n + 1,) or rowptr[0] != 0 or np.any(np.diff(rowptr) < 0):
        raise CsrcError("bad row pointer")
    nnz = int(rowptr[-1])
    if col.shape[0] != nnz or val.shape[0] != nnz:
        raise CsrcError("bad array lengths")
    if nnz and (col.min() < 0 or col.max() >= n):
        raise CsrcError("column index out of range")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    key = rows * n + col
    order = np.argsort(key, kind="stable")
    key = key[order]
    if nnz and np.any(key[1:] == key[:-1]):
        raise CsrcError("duplicate entry")
    rows = rows[order]
    col = col[order]
    val = val[order]
    mirror = col * n + rows
    present = np.isin(mirror, key, assume_unique=False)
    if not np.all(present):
        if not pad:
            raise CsrcError("pattern is not structurally symmetric")
        # add an explicit zero at each missing mirror position
        mr = col[~present]
        mc = rows[~present]
        rows = np.concatenate([rows, mr])
        col = np.concatenate([col, mc])
        val = np.concatenate([val, np.zeros(mr.shape[0])])
        key = rows * n + col
        order = np.argsort(key, kind="stable")
        rows, col, val = rows[order], col[order], val[order]
    ad = np.zeros(n, dtype=np.float64)
    d = rows == col
    ad[rows[d]] = val[d]
    lo = col < rows
    # lower entries in (row, col) order: row-wise CSR of A_L
    l_rows, l_cols, l_vals = rows[lo], col[lo], val[lo]
    # upper entries (r, c), c > r, ordered by their mirror (c, r): column-wise A_U
    up = col > rows
    u_rows, u_cols, u_vals = rows[up], col[up], val[up]
    uo = np.argsort(u_cols * n + u_rows, kind="stable")
    assert np.array_equal(u_cols[uo], l_rows) and np.array_equal(u_rows[uo], l_cols)
    ia = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(l_rows, minlength=n), out=ia[1:])
    k = int(ia[-1])
    if k >= 2**31:
        raise CsrcError("too many entries for 32-bit indices")
    return {
        "n": int(n), "k": k,
        "ia": ia.astype(np.int32), "ja": l_cols.astype(np.int32),
        "ad": ad, "al": l_vals.copy(), "au": u_vals[uo].copy(),
    }


def csrc_to_dense(c):
    """Dense matrix of a CSRC triple (tiny cases only)."""
    n = c["n"]
    A = np.zeros((n, n))
    A[np.arange(n), np.arange(n)] = c["ad"]
    for i in range(n):
        for q in range(c["ia"][i], c["ia"][i + 1]):
            j = c["ja"][q]
            A[i, j] = c["al"][q]
            A[j, i] = c["au"][q]
    return A


# --------------------------------------------------------------------------
# Product (Sec. 2 splitting) and transpose (Sec. 5)
# --------------------------------------------------------------------------

def _vals(c, name, override):
    v = override.get(name, c[name])
    return np.ascontiguousarray(v, dtype=np.float64)


def spmv(c, x, **override):
    """y = A x = (A_D + A_L + A_U) x, term by term (C oracle, FP64, no FMA)."""
    n = c["n"]
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    ia = np.ascontiguousarray(c["ia"], dtype=np.int32)
    ja = np.ascontiguousarray(c["ja"], dtype=np.int32)
    ad, al, au = (_vals(c, s, override) for s in ("ad", "al", "au"))
    lib().oracle_csrc_spmv(n, _p(ia), _p(ja), _p(ad), _p(al), _p(au), _p(x), _p(y))
    return y


def spmv_t(c, x, **override):
    """y = A^T x: the same splitting with al and au exchanged (Sec. 5)."""
    n = c["n"]
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    ia = np.ascontiguousarray(c["ia"], dtype=np.int32)
    ja = np.ascontiguousarray(c["ja"], dtype=np.int32)
    ad, al, au = (_vals(c, s, override) for s in ("ad", "al", "au"))
    lib().oracle_csrc_spmv_t(n, _p(ia), _p(ja), _p(ad), _p(al), _p(au), _p(x), _p(y))
    return y


def spmm(c, X, **override):
    """Y = A X for an n x r row-major block, column by column."""
    n = c["n"]
    X = np.ascontiguousarray(X, dtype=np.float64)
    r = X.shape[1]
    Y = np.zeros((n, r), dtype=np.float64)
    ia = np.ascontiguousarray(c["ia"], dtype=np.int32)
    ja = np.ascontiguousarray(c["ja"], dtype=np.int32)
    ad, al, au = (_vals(c, s, override) for s in ("ad", "al", "au"))
    lib().oracle_csrc_spmm(n, _p(ia), _p(ja), _p(ad), _p(al), _p(au), r, _p(X), r, _p(Y), r)
    return Y


def split_rect(n, m, rowptr, col, val):
    """Sec. 2.1: an n x m matrix (m >= n) as A_S + A_R.  A_S (n x n) holds
    the entries of columns < n and goes to CSRC; A_R holds those of columns
    >= n as CSR (``iar`` int32[n+1], ``jar`` int32 global column indices,
    ``ar`` float64), each row in input order.  Returns (CSR of A_S as
    (rowptr, col, val), dict(n, m, kr, iar, jar, ar))."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    val = np.asarray(val, dtype=np.float64)
    if m < n or rowptr.shape != (n + 1,) or np.any(col < 0) or np.any(col >= m):
        raise CsrcError("bad rectangular matrix")
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    sq = col < n
    s_rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[sq], minlength=n), out=s_rowptr[1:])
    iar = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows[~sq], minlength=n), out=iar[1:])
    r = {"n": n, "m": m, "kr": int(iar[-1]), "iar": iar.astype(np.int32),
         "jar": col[~sq].astype(np.int32), "ar": val[~sq].copy()}
    return (s_rowptr, col[sq].astype(np.int32), val[sq].copy()), r


def spmv_rect(c, r, x, **override):
    """y = A x for A = A_S + A_R (Fig. 2b): the square CSRC product on x[:n],
    then each row's auxiliary CSR entries gathered from the whole x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n = c["n"]
    y = spmv(c, x[:n], **override)
    ar = override.get("ar", r["ar"])
    iar, jar = r["iar"], r["jar"]
    for i in range(n):
        t = y[i]
        for q in range(iar[i], iar[i + 1]):
            t += ar[q] * x[jar[q]]
        y[i] = t
    return y


def spmv_rect_t(c, r, x, **override):
    """y = A^T x (y has m entries): A_S^T x on the first n, and each entry
    of A_R scattered into y[jar] (the transpose of the auxiliary CSR)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    n, m = c["n"], r["m"]
    y = np.zeros(m, dtype=np.float64)
    y[:n] = spmv_t(c, x, **override)
    ar = override.get("ar", r["ar"])
    iar, jar = r["iar"], r["jar"]
    for i in range(n):
        for q in range(iar[i], iar[i + 1]):
            y[jar[q]] += ar[q] * x[i]
    return y


def spmv_py(c, x, transpose=False):
    """Pure-Python product for tiny inputs, from A = A_D + A_L + A_U
    (Sec. 2): the diagonal term, then every stored lower entry a_ij x_j into
    y_i, then every mirrored upper entry a_ji x_i into y_j (same order and
    rounding as the C oracle).  The transpose exchanges al and au (Sec. 5)."""
    n = c["n"]
    ia, ja, ad = c["ia"], c["ja"], c["ad"]
    al, au = (c["au"], c["al"]) if transpose else (c["al"], c["au"])
    y = [float(ad[i]) * float(x[i]) for i in range(n)]
    for i in range(n):
        for q in range(int(ia[i]), int(ia[i + 1])):
            y[i] = y[i] + float(al[q]) * float(x[int(ja[q])])
    for i in range(n):
        for q in range(int(ia[i]), int(ia[i + 1])):
            j = int(ja[q])
            y[j] = y[j] + float(au[q]) * float(x[i])
    return np.array(y)


# --------------------------------------------------------------------------
# Setup: colouring (Sec. 3.2), partition and effective ranges (Sec. 3.1)
# --------------------------------------------------------------------------

WRITE_SET = 0
DISTANCE2 = 1


def color(c, criterion=WRITE_SET):
    """Greedy first-fit colouring, rows in ascending order (C oracle)."""
    n = c["n"]
    ia = np.ascontiguousarray(c["ia"], dtype=np.int32)
    ja = np.ascontiguousarray(c["ja"], dtype=np.int32)
    out = np.zeros(n, dtype=np.int32)
    nc = lib().oracle_csrc_color(n, _p(ia), _p(ja), criterion, _p(out))
    if nc < 0:
        raise MemoryError("oracle colouring")
    return out, int(nc)


def write_set(c, i):
    """W(i) = {i} U {ja[k] : k in row i}: the entries of y row i's loop writes."""
    return {i} | set(int(j) for j in c["ja"][c["ia"][i]:c["ia"][i + 1]])


def conflicts_py(c, criterion=WRITE_SET):
    """Conflict sets by definition (tiny inputs): list of sets per row."""
    n = c["n"]
    W = [write_set(c, i) for i in range(n)]
    if criterion == WRITE_SET:
        return [set(r for r in range(n) if r != i and W[i] & W[r]) for i in range(n)]
    nb = [set() for _ in range(n)]
    for i in range(n):
        for j in W[i] - {i}:
            nb[i].add(j)
            nb[j].add(i)
    return [set(r for r in range(n) if r != i and (r in nb[i] or nb[i] & nb[r])) for i in range(n)]


def color_py(c, criterion=WRITE_SET):
    """Greedy first-fit colouring from the conflict sets (tiny inputs)."""
    conf = conflicts_py(c, criterion)
    col = []
    for i in range(c["n"]):
        used = {col[r] for r in conf[i] if r < i}
        k = 0
        while k in used:
            k += 1
        col.append(k)
    return np.array(col, dtype=np.int32), (max(col) + 1 if col else 0)


def row_weights(ia):
    """Work of row i's loop: 2 per stored lower pair (al and au) + 1 (diagonal)."""
    ia = np.asarray(ia, dtype=np.int64)
    return 2 * np.diff(ia) + 1


def partition(ia, parts):
    """nnz-guided partition into ``parts`` contiguous row blocks (Sec. 3.1).

    Block b ends at the first row i whose prefix work C(i) = sum_{r<i} w_r
    reaches (b+1)/parts of the total.  Returns the ``parts + 1`` boundaries.
    """
    w = row_weights(ia)
    n = w.shape[0]
    C = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(w, out=C[1:])
    total = int(C[-1])
    b = np.arange(1, parts, dtype=np.int64)
    # smallest i with C(i) * parts >= b * total
    s = np.searchsorted(C * parts, b * total, side="left")
    return np.concatenate([[0], s, [n]]).astype(np.int64)


def cap_rows(bounds, max_rows):
    """Split every block of more than ``max_rows`` rows into m = ceil(rows /
    max_rows) pieces with boundaries r0 + floor(p * rows / m), p = 0..m.

    (A GPU tile keeps per-row state of its block on chip, so its row count
    needs a bound; blocks within the bound are unchanged.)
    """
    out = [int(bounds[0])]
    for b in range(len(bounds) - 1):
        r0, r1 = int(bounds[b]), int(bounds[b + 1])
        rows = r1 - r0
        m = max(1, -(-rows // max_rows))
        for p in range(1, m + 1):
            out.append(r0 + (p * rows) // m)
    return np.array(out, dtype=np.int64)


def drop_empty(bounds):
    """The non-empty blocks of a partition: boundaries with repeats removed.

    (With more blocks than rows, or rows heavier than a block's share, the
    partition has empty blocks; a GPU tile is a non-empty block.)
    """
    bounds = np.asarray(bounds, dtype=np.int64)
    if bounds.shape[0] < 2:
        return bounds
    keep = np.concatenate([[True], bounds[1:] != bounds[:-1]])
    return bounds[keep]


def partition_for_target(ia, target, max_rows=2048):
    """Partition with ceil(total work / target) blocks, then the row cap;
    the tiles are the non-empty blocks."""
    total = int(row_weights(ia).sum())
    parts = max(1, -(-total // int(target)))
    return drop_empty(cap_rows(partition(ia, parts), max_rows))


def out_of_tile_targets(c, r0, r1):
    """Sorted rows below the block [r0, r1) that the block's loops write into.

    With the block's own rows this is the block's effective range (Sec. 3.1).
    """
    lo, hi = int(c["ia"][r0]), int(c["ia"][r1])
    t = np.unique(c["ja"][lo:hi])
    return t[t < r0]


def color_blocks(write_sets):
    """Colour classes of row blocks with a bounded stride (the refinement of
    the colourful method proposed in Sec. 5): block b writes the rows in
    ``write_sets[b]``; blocks b and d conflict iff those sets meet.  Greedy
    first-fit in ascending block order, as in Sec. 3.2 for rows.  Returns
    (colour per block, number of colours)."""
    sets = [set(int(r) for r in w) for w in write_sets]
    col = []
    for b, wb in enumerate(sets):
        used = {col[d] for d in range(b) if wb & sets[d]}
        k = 0
        while k in used:
            k += 1
        col.append(k)
    return np.array(col, dtype=np.int32), (max(col) + 1 if col else 0)


# --------------------------------------------------------------------------
# Reduced precision: rounding and error bounds
# --------------------------------------------------------------------------

def to_f32(a):
    """Round to nearest even FP32 (IEEE conversion)."""
    return np.asarray(a, dtype=np.float64).astype(np.float32)


def to_bf16_bits(a):
    """bfloat16 bits of RNE(RNE_fp32(a)); NaN stays a quiet NaN."""
    f = to_f32(a)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16))
    r = np.where(nan, (u >> np.uint64(16)) | np.uint64(0x40), r)
    return r.astype(np.uint16)


def bf16_to_f64(bits):
    return (np.asarray(bits, dtype=np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def dequantize(a, dtype):
    """Values a stored copy in ``dtype`` represents, as float64."""
    if dtype == "f64":
        return np.asarray(a, dtype=np.float64)
    if dtype == "f32":
        return to_f32(a).astype(np.float64)
    if dtype == "bf16":
        return bf16_to_f64(to_bf16_bits(a))
    raise ValueError(dtype)


UNIT_ROUNDOFF = {"f64": 2.0**-53, "f32": 2.0**-24, "bf16": 2.0**-8}


def gamma(m, u):
    """gamma_m = m u / (1 - m u) (Higham, Accuracy and Stability, Sec. 3.1)."""
    m = np.asarray(m, dtype=np.float64)
    return m * u / (1.0 - m * u)


def row_terms(c):
    """Number of products summed into each y_i: diagonal + lower + upper."""
    n = c["n"]
    cnt = np.ones(n, dtype=np.int64)
    cnt += np.diff(c["ia"].astype(np.int64))
    cnt += np.bincount(c["ja"], minlength=n)
    return cnt


def abs_product(c, x, transpose=False, **override):
    """|A| |x| (FP64): the scale of every error bound."""
    cc = dict(c)
    for s in ("ad", "al", "au"):
        cc[s] = np.abs(override.get(s, c[s]))
    f = spmv_t if transpose else spmv
    return f(cc, np.abs(x))


def accumulation_bound(c, x, u_acc, transpose=False, **override):
    """|y_hat - y| <= gamma_{m_i}(u_acc) (|A||x|)_i for any summation order."""
    return gamma(row_terms(c), u_acc) * abs_product(c, x, transpose, **override)

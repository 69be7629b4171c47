"""Matrix values and source vectors for generated patterns.

Off-diagonal ``a_ij`` is uniform on [-1, 1), drawn independently for the
ordered pair of *natural* ids ``(orig[i], orig[j])`` (so ``a_ij`` and ``a_ji``
are independent: the matrix is numerically non-symmetric).  The diagonal is
``1 + sum_{j != i} |a_ij|`` over the stored row, which makes the matrix strictly
diagonally dominant.  ``kind="int"`` draws every entry (diagonal included) and
every vector element as an integer in [-8, 8]: sums of such products are exact
in any order in binary floating point, down to bfloat16 storage.
``kind="sym"`` keys the off-diagonals on the unordered pair (numerically
symmetric matrix).
"""

import numpy as np

from .rng import uniform_pm1, randint_pm


def fill_values(a, seed, kind="uniform"):
    rows = a.rows()
    cols = a.col.astype(np.int64)
    oi = a.orig[rows]
    oj = a.orig[cols]
    diag = rows == cols
    if kind == "sym":
        lo = np.minimum(oi, oj)
        hi = np.maximum(oi, oj)
        v = uniform_pm1(seed, 1, hi, lo)
    elif kind == "int":
        v = randint_pm(seed, 1, 8, oi, oj)
    else:
        v = uniform_pm1(seed, 1, oi, oj)
    if kind == "int":
        v[diag] = randint_pm(seed, 2, 8, oi[diag])
    else:
        v[diag] = 0.0
        rowabs = np.bincount(rows, weights=np.abs(v), minlength=a.n)
        v[diag] = 1.0 + rowabs[rows[diag]]
    a.val = v
    a.meta["values"] = {"seed": seed, "kind": kind}
    return a


def vector(a_or_orig, seed, kind="uniform"):
    """Source vector keyed by natural id: x[i] = f(seed, orig[i])."""
    orig = a_or_orig.orig if hasattr(a_or_orig, "orig") else np.asarray(a_or_orig)
    if kind == "int":
        return randint_pm(seed, 3, 8, orig)
    return uniform_pm1(seed, 3, orig)


def block_vector(a_or_orig, r, seed, kind="uniform"):
    """n x r row-major block of right-hand sides: X[i, c] = f(seed, orig[i], c)."""
    orig = a_or_orig.orig if hasattr(a_or_orig, "orig") else np.asarray(a_or_orig)
    oi = np.repeat(orig, r)
    c = np.tile(np.arange(r, dtype=np.int64), len(orig))
    if kind == "int":
        v = randint_pm(seed, 4, 8, oi, c)
    else:
        v = uniform_pm1(seed, 4, oi, c)
    return v.reshape(len(orig), r)

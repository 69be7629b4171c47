"""Shared test helpers: matrix recipes, error metrics."""

import numpy as np

from oracle import reference as R
from synth import patterns as P, workloads as W
from synth.values import fill_values, vector


def rel_inf(y, ref):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = np.max(np.abs(y - ref)) if y.size else 0.0
    s = np.max(np.abs(ref)) if ref.size else 0.0
    return d / s if s > 0 else d


def with_x(a, seed=3, kind="uniform"):
    return a, vector(a, seed, kind)


def arrow(n, seed=1, kind="uniform"):
    """Row 0 and column 0 dense plus the diagonal: one very long row at the end
    after reversing (row n-1 stores n-1 lower entries)."""
    rows = [0] * n + list(range(1, n)) + list(range(1, n))
    cols = list(range(n)) + [0] * (n - 1) + list(range(1, n))
    key = np.array(rows, np.int64) * n + np.array(cols, np.int64)
    key = np.unique(key)
    r, c = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    a = P.CSR(n=n, rowptr=rp, col=c.astype(np.int32), orig=np.arange(n, dtype=np.int64), meta={"kind": "arrow"})
    a = P.reorder(a, np.arange(n)[::-1].copy())
    fill_values(a, seed, kind)
    return a


def diagonal_only(n, seed=1, kind="uniform"):
    a = P.banded(n, 0, 1.0, 0)
    fill_values(a, seed, kind)
    return a


def empty_rows(n=300, seed=1, kind="uniform"):
    """Pattern with isolated rows and a missing diagonal on every third row."""
    rng = np.random.default_rng(seed)
    li = rng.integers(1, n, 200)
    lj = (li * rng.random(200)).astype(np.int64)
    keep = lj < li
    li, lj = li[keep], lj[keep]
    d = np.arange(n)
    d = d[d % 3 != 0]
    r = np.concatenate([d, li, lj])
    c = np.concatenate([d, lj, li])
    key = np.unique(r * n + c)
    r, c = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=rp[1:])
    a = P.CSR(n=n, rowptr=rp, col=c.astype(np.int32), orig=np.arange(n, dtype=np.int64), meta={"kind": "ragged"})
    fill_values(a, seed, kind)
    return a


def small_cases(kind="uniform"):
    """(name, CSR, x) triples spanning several tiles and ragged tails."""
    out = []
    a, x = W.quad64(kind=kind)
    out.append(("quad64", a, x))
    for o in ("natural", "random", "rcm"):
        a, x = W.hex_mesh(17, o, kind=kind)
        out.append((f"hex17_{o}", a, x))
    a, x = W.tet_mesh(7, kind=kind)
    out.append(("tet7x3", a, x))
    a = fill_values(P.banded(7001, 33, 0.4, 3), 4, kind)
    out.append(("banded7001", a, vector(a, 5, kind)))
    a = fill_values(P.reorder(P.power_law(6000, 20.0, 2.5, 7), P.random_order(6000, 9)), 6, kind)
    out.append(("powerlaw6000", a, vector(a, 7, kind)))
    a = arrow(1500, kind=kind)
    out.append(("arrow1500", a, vector(a, 8, kind)))
    a = diagonal_only(777, kind=kind)
    out.append(("diag777", a, vector(a, 9, kind)))
    a = empty_rows(kind=kind)
    out.append(("ragged300", a, vector(a, 10, kind)))
    a = fill_values(P.q1_quad(1, 1), 1, kind)
    out.append(("n1", a, vector(a, 11, kind)))
    return out


def oracle_csrc(a):
    return R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)

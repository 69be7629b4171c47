"""The selector's 12 structural features, by definition -- TEST INFRASTRUCTURE.

Row lengths count the diagonal once per row plus the lower and mirrored upper
entries; nnz = 2k + n.  Written from the definitions in the library's
header; pinned in tests/test_lib_host.py against hand-computed values on a
small pattern, and used there to check csrc_features on larger ones.
"""

import numpy as np

from . import reference as R


def features(c, vdtype="f64", ncolors=None):
    n, k = c["n"], c["k"]
    ia = c["ia"].astype(np.int64)
    ja = c["ja"].astype(np.int64)
    rows = np.repeat(np.arange(n), np.diff(ia))
    nnz = 2 * k + n
    length = 1 + np.bincount(rows, minlength=n) + np.bincount(ja, minlength=n)
    writers = 1 + np.bincount(ja, minlength=n)
    d = rows - ja
    mean = nnz / n
    if ncolors is None:
        ncolors = R.color(c, R.WRITE_SET)[1]
    lower = np.diff(ia)
    block3 = n % 3 == 0 and n >= 3
    if block3:
        l0, l1, l2 = lower[0::3], lower[1::3], lower[2::3]
        block3 = bool(np.all(l1 == l0 + 1) and np.all(l2 == l0 + 2) and np.all(l0 % 3 == 0))
    vb = {"f64": 8, "f32": 4, "bf16": 2}[vdtype]
    xb = 8 if vdtype == "f64" else 4
    ws = 4.0 * (n + 1) + k * (4 + 2 * vb) + n * vb + n * 2 * xb
    return np.array([
        np.log2(n + 1.0),
        np.log2(nnz + 1.0),
        mean,
        np.mean((length - mean) ** 2),
        length.max() / mean,
        (d.max() if k else 0) / n,
        (d.mean() / n) if k else 0.0,
        (np.mean(d < 64)) if k else 1.0,
        np.log2(1.0 + writers.max()),
        ncolors / 32.0,
        np.log2(ws / (256.0 * 1024 * 1024)),
        1.0 if block3 else 0.0,
    ])

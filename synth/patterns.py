"""Structurally symmetric sparsity patterns shaped like finite element matrices.

Every generator returns a :class:`CSR` whose rows are sorted by column and whose
pattern is structurally symmetric (``(i, j)`` stored iff ``(j, i)`` stored).
``orig`` records, for each row in the current numbering, the id of the row in
the generator's natural numbering; values are keyed on those ids so that a
renumbered matrix represents the same operator ``P A P^T``.
"""

from dataclasses import dataclass, field
import itertools

import numpy as np

from .rng import uniform01, splitmix64


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray           # int64, n + 1
    col: np.ndarray              # int32, nnz, sorted within each row
    val: np.ndarray = None       # float64, nnz (filled by values.fill_values)
    orig: np.ndarray = None      # int64, n: natural id of each row
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def rows(self):
        """Row index of every stored entry (int64, nnz)."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.rowptr))


def stencil_offsets_2d(points):
    """Offsets of the 5-point or 9-point 2D stencil."""
    if points == 9:
        return [(dx, dy, 0) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    if points == 5:
        return [(0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0)]
    raise ValueError(points)


def stencil_offsets_3d(points):
    """Offsets of the 7-point, 15-point (Kuhn/Freudenthal) or 27-point stencil."""
    if points == 27:
        return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    if points == 7:
        return [(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]
    if points == 15:
        # Kuhn (Freudenthal) split of every cube into 6 tetrahedra that share
        # the (0,0,0)-(1,1,1) diagonal: the mesh edges are +-sum_{i in S} e_i
        # for each non-empty S of {x, y, z}, so each node has 14 neighbours.
        vecs = []
        for s in range(1, 8):
            v = ((s >> 0) & 1, (s >> 1) & 1, (s >> 2) & 1)
            vecs.append(v)
            vecs.append(tuple(-c for c in v))
        return vecs + [(0, 0, 0)]
    raise ValueError(points)


def grid_stencil(dims, offsets):
    """Pattern of a stencil on a structured grid, natural numbering.

    Node ``(x, y, z)`` has id ``x + nx*(y + ny*z)``.  The pattern row of a node
    holds every in-grid node at one of ``offsets``.  The offsets list must be
    closed under negation (so the pattern is structurally symmetric).
    """
    nx, ny, nz = (tuple(dims) + (1, 1))[:3]
    n = nx * ny * nz
    lin = lambda o: o[0] + nx * (o[1] + ny * o[2])
    offs = sorted(set(tuple(o) for o in offsets), key=lin)
    assert all(tuple(-c for c in o) in offs for o in offs), "offsets not symmetric"
    idx = np.arange(n, dtype=np.int64)
    x = idx % nx
    y = (idx // nx) % ny
    z = idx // (nx * ny)
    masks = []
    for dx, dy, dz in offs:
        m = np.ones(n, dtype=bool)
        if dx:
            m &= (x + dx >= 0) & (x + dx < nx)
        if dy:
            m &= (y + dy >= 0) & (y + dy < ny)
        if dz:
            m &= (z + dz >= 0) & (z + dz < nz)
        masks.append(m)
    counts = np.zeros(n, dtype=np.int64)
    for m in masks:
        counts += m
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = np.empty(int(rowptr[-1]), dtype=np.int32)
    pos = rowptr[:-1].copy()
    # Offsets are visited in ascending linear offset, so each row is filled in
    # ascending column order.
    for o, m in zip(offs, masks):
        r = np.nonzero(m)[0]
        col[pos[r]] = (r + lin(o)).astype(np.int32)
        pos[r] += 1
    return CSR(n=n, rowptr=rowptr, col=col, orig=idx.copy(),
               meta={"kind": "stencil", "dims": (nx, ny, nz), "points": len(offs)})


def q1_quad(nx, ny):
    """Bilinear quadrilateral mesh of nx x ny nodes: the 9-point pattern."""
    a = grid_stencil((nx, ny, 1), stencil_offsets_2d(9))
    a.meta.update(kind="q1_quad")
    return a


def q1_hex(nx, ny, nz):
    """Trilinear hexahedral mesh of nx x ny x nz nodes: the 27-point pattern."""
    a = grid_stencil((nx, ny, nz), stencil_offsets_3d(27))
    a.meta.update(kind="q1_hex")
    return a


def block_expand(a, b):
    """Replace every entry of a node pattern by a dense b x b block.

    Degree of freedom ``c`` of node ``v`` gets id ``b*v + c`` (interleaved).
    """
    n = a.n
    cnt = np.diff(a.rowptr)
    # expanded column list of each node row: (b*col + c) for each col, c
    colx = (b * a.col.astype(np.int64)[:, None] + np.arange(b)[None, :]).ravel()
    seg_start = b * a.rowptr[:-1]
    seg_len = b * cnt
    rowcnt = np.repeat(seg_len, b)
    rowptr = np.zeros(b * n + 1, dtype=np.int64)
    np.cumsum(rowcnt, out=rowptr[1:])
    starts = np.repeat(seg_start, b)
    # gather index for every output entry: starts[row] + position in row
    rows = np.repeat(np.arange(b * n, dtype=np.int64), rowcnt)
    within = np.arange(int(rowptr[-1]), dtype=np.int64) - rowptr[:-1][rows]
    col = colx[starts[rows] + within].astype(np.int32)
    orig = (b * a.orig[:, None] + np.arange(b)[None, :]).ravel()
    meta = dict(a.meta)
    meta.update(block=b)
    return CSR(n=b * n, rowptr=rowptr, col=col, orig=orig, meta=meta)


def kuhn_tet(nx, ny, nz, dof=3):
    """Tetrahedral mesh (6 Kuhn tets per grid cube) with ``dof`` unknowns per node.

    Node coordinates may be jittered by a caller; the pattern depends only on
    the mesh connectivity, which jitter does not change.
    """
    a = grid_stencil((nx, ny, nz), stencil_offsets_3d(15))
    a.meta.update(kind="kuhn_tet")
    if dof > 1:
        a = block_expand(a, dof)
    return a


def _from_lower_pairs(n, li, lj, kind, meta=None):
    """Symmetric pattern with full diagonal from strictly-lower pairs (li > lj)."""
    d = np.arange(n, dtype=np.int64)
    r = np.concatenate([d, li, lj])
    c = np.concatenate([d, lj, li])
    key = r * n + c
    key = np.unique(key)
    r = key // n
    c = key % n
    counts = np.bincount(r, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    m = {"kind": kind}
    if meta:
        m.update(meta)
    return CSR(n=n, rowptr=rowptr, col=c.astype(np.int32), orig=d.copy(), meta=m)


def banded(n, half_bw, fill, seed):
    """Random banded pattern: pair (i, i-o), 1 <= o <= half_bw, kept w.p. ``fill``."""
    li = []
    lj = []
    for o in range(1, half_bw + 1):
        i = np.arange(o, n, dtype=np.int64)
        keep = uniform01(seed, 7, i, np.full_like(i, o)) < fill
        li.append(i[keep])
        lj.append(i[keep] - o)
    li = np.concatenate(li) if li else np.zeros(0, np.int64)
    lj = np.concatenate(lj) if lj else np.zeros(0, np.int64)
    return _from_lower_pairs(n, li, lj, "banded", {"half_bw": half_bw, "fill": fill})


def power_law(n, mean_deg, exponent, seed):
    """Chung-Lu style random graph with power-law expected degrees.

    Node weights ``w_i ~ (i + i0)^(-1/(exponent-1))`` are scaled to mean
    ``mean_deg``; ``n*mean_deg/2`` edge endpoints are drawn independently with
    probability proportional to the weights (inverse-CDF on a counter-based
    uniform), self loops and repeats dropped.  Numbering is natural by weight
    rank; callers renumber at random.
    """
    i = np.arange(n, dtype=np.float64)
    w = (i + 1.0) ** (-1.0 / (exponent - 1.0))
    w *= mean_deg / w.mean()
    w = np.minimum(w, n - 1)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m = int(n * mean_deg / 2)
    e = np.arange(m, dtype=np.int64)
    a = np.searchsorted(cdf, uniform01(seed, 11, e), side="right")
    b = np.searchsorted(cdf, uniform01(seed, 12, e), side="right")
    a = np.minimum(a, n - 1)
    b = np.minimum(b, n - 1)
    keep = a != b
    li = np.maximum(a[keep], b[keep])
    lj = np.minimum(a[keep], b[keep])
    return _from_lower_pairs(n, li, lj, "power_law", {"mean_deg": mean_deg, "exponent": exponent})


def reorder(a, order):
    """Renumber so that new row ``r`` is old row ``order[r]`` (P A P^T)."""
    n = a.n
    order = np.asarray(order, dtype=np.int64)
    pos = np.empty(n, dtype=np.int64)
    pos[order] = np.arange(n, dtype=np.int64)
    old_rows = a.rows()
    nr = pos[old_rows]
    nc = pos[a.col.astype(np.int64)]
    key = nr * n + nc
    perm = np.argsort(key, kind="stable")
    counts = np.bincount(nr, minlength=n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = nc[perm].astype(np.int32)
    val = None if a.val is None else a.val[perm]
    meta = dict(a.meta)
    return CSR(n=n, rowptr=rowptr, col=col, val=val, orig=a.orig[order], meta=meta)


def permute(a, order):
    return reorder(a, order)


def random_order(n, seed):
    """Seeded uniform random permutation: rows sorted by a counter-based
    uniform key (53 random bits each; ties broken by index)."""
    u = uniform01(seed, 21, np.arange(n, dtype=np.int64))
    return np.argsort(u, kind="stable").astype(np.int64)


def rcm_order(a):
    """Reverse Cuthill-McKee numbering from scipy's csgraph routine."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import reverse_cuthill_mckee
    m = sp.csr_matrix((np.ones(a.nnz, dtype=np.int8), a.col, a.rowptr), shape=(a.n, a.n))
    return np.asarray(reverse_cuthill_mckee(m, symmetric_mode=True), dtype=np.int64)

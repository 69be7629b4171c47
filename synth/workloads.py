"""Named synthetic workloads (pattern + values + vectors), all seeded.

* ``quad64``   2D bilinear quad mesh, 64 x 64 nodes, 9-point pattern (n=4096).
* ``hex100``   3D trilinear hex mesh, 100^3 nodes, 27-point pattern (n=1e6),
               natural / seeded random / RCM numbering.
* ``tet80x3``  Kuhn tetrahedral mesh on 80^3 nodes, 3 dofs per node (n=1.536e6).
* ``batch256`` 256 matrices of uneven size (n log-uniform 1e3..2e5, 9-point or
               27-point) each with 1..32 right-hand sides.
* ``family``   the selector's training family (stencils, banded, 3x3-block FEM,
               power-law graphs).
"""

import math

import numpy as np

from . import patterns as P
from .rng import uniform01
from .values import fill_values, vector, block_vector


def quad64(kind="uniform", side=64):
    a = P.q1_quad(side, side)
    fill_values(a, 1001, kind)
    x = vector(a, 1101, kind)
    a.meta["name"] = f"quad{side}"
    return a, x


def hex_mesh(side=100, ordering="natural", kind="uniform"):
    a = P.q1_hex(side, side, side)
    fill_values(a, 1002, kind)
    if ordering == "random":
        a = P.reorder(a, P.random_order(a.n, 2002))
    elif ordering == "rcm":
        a = P.reorder(a, P.rcm_order(a))
    elif ordering != "natural":
        raise ValueError(ordering)
    x = vector(a, 1102, kind)
    a.meta["name"] = f"hex{side}_{ordering}"
    a.meta["ordering"] = ordering
    return a, x


def rect_mesh(side=17, extra=None, kind="uniform"):
    """An n x m matrix of the overlapping-subdomain kind (Sec. 2.1): the
    27-point mesh of side^3 nodes (its own rows and columns) plus couplings
    of the nodes of the top face (z = side - 1) to `extra` overlap nodes
    numbered n .. m-1 (each top node couples to the overlap nodes above it
    and its grid neighbours').  Returns (CSR n x m, x of m values)."""
    a = P.q1_hex(side, side, side)
    fill_values(a, 1005, kind)
    n = a.n
    ex = extra if extra is not None else side * side
    rows, cols = [], []
    top = np.arange(n - side * side, n)
    for d in (-1, 0, 1):
        tgt = (top - (n - side * side)) + d
        ok = (tgt >= 0) & (tgt < ex)
        rows.append(top[ok])
        cols.append(n + tgt[ok])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    u = uniform01(1006, 5, rows.astype(np.int64) * (n + ex) + cols)
    vals = np.round(16 * u - 8) if kind == "int" else 2.0 * u - 1.0
    base_rows = np.repeat(np.arange(n), np.diff(a.rowptr))
    all_rows = np.concatenate([base_rows, rows])
    all_cols = np.concatenate([a.col.astype(np.int64), cols])
    all_vals = np.concatenate([a.val, vals])
    order = np.lexsort((all_cols, all_rows))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(all_rows, minlength=n), out=rowptr[1:])
    m = n + ex
    ux = uniform01(1105, 6, np.arange(m, dtype=np.int64))
    x = np.round(16 * ux - 8) if kind == "int" else 2.0 * ux - 1.0
    return (n, m, rowptr, all_cols[order].astype(np.int32), all_vals[order]), x


def tet_mesh(side=80, dof=3, kind="uniform"):
    a = P.kuhn_tet(side, side, side, dof)
    fill_values(a, 1003, kind)
    x = vector(a, 1103, kind)
    a.meta["name"] = f"tet{side}x{dof}"
    return a, x


def batch_spec(m, n_lo=1e3, n_hi=2e5):
    """Shape of batch member m: (family, grid dims, r)."""
    s = 40000 + m
    u = uniform01(s, 31, np.arange(3, dtype=np.int64))
    nstar = math.exp(math.log(n_lo) + u[0] * (math.log(n_hi) - math.log(n_lo)))
    r = 1 + int(u[2] * 32)
    if u[1] < 0.5:
        side = max(2, int(round(math.sqrt(nstar))))
        return ("quad9", (side, side, 1), r)
    side = max(2, int(round(nstar ** (1.0 / 3.0))))
    return ("hex27", (side, side, side), r)


def batch_member(m, kind="uniform", n_lo=1e3, n_hi=2e5):
    fam, dims, r = batch_spec(m, n_lo, n_hi)
    if fam == "quad9":
        a = P.q1_quad(dims[0], dims[1])
    else:
        a = P.q1_hex(*dims)
    fill_values(a, 40000 + m, kind)
    X = block_vector(a, r, 41000 + m, kind)
    a.meta["name"] = f"batch{m}_{fam}_{a.n}"
    return a, X


FAMILIES = ("stencil", "banded", "fem3", "power")


def family_spec(m, n_lo=1e4, n_hi=2e6, nnz_cap=None):
    """Spec of selector-family member m (all choices from counter uniforms)."""
    s = 50000 + m
    u = uniform01(s, 41, np.arange(8, dtype=np.int64))
    fam = FAMILIES[int(u[0] * 4) % 4]
    n = int(math.exp(math.log(n_lo) + u[1] * (math.log(n_hi) - math.log(n_lo))))
    spec = {"m": m, "family": fam, "n": n, "seed": s}
    if fam == "stencil":
        pts = (5, 9, 7, 27)[int(u[2] * 4) % 4]
        spec["points"] = pts
        spec["ordering"] = ("natural", "random", "rcm")[int(u[3] * 3) % 3]
    elif fam == "banded":
        spec["half_bw"] = int(round(math.exp(math.log(2) + u[2] * (math.log(512) - math.log(2)))))
        spec["fill"] = 0.05 + 0.95 * float(u[3])
    elif fam == "fem3":
        spec["ordering"] = ("natural", "random", "rcm")[int(u[3] * 3) % 3]
    else:
        spec["mean_deg"] = 4.0 + 196.0 * float(u[2]) ** 2
        spec["exponent"] = 2.5
    if nnz_cap is not None:
        est = _nnz_estimate(spec)
        if est > nnz_cap:
            spec["n"] = max(1000, int(spec["n"] * nnz_cap / est))
    return spec


def _nnz_estimate(spec):
    n = spec["n"]
    f = spec["family"]
    if f == "stencil":
        return n * spec["points"]
    if f == "banded":
        return n * (1 + 2 * spec["half_bw"] * spec["fill"])
    if f == "fem3":
        return n * 45
    return n * (1 + spec["mean_deg"])


def family_member(spec, kind="uniform"):
    f = spec["family"]
    n = spec["n"]
    s = spec["seed"]
    order = spec.get("ordering", "natural")
    if f == "stencil":
        pts = spec["points"]
        if pts in (5, 9):
            side = max(2, int(round(math.sqrt(n))))
            a = P.grid_stencil((side, side, 1), P.stencil_offsets_2d(pts))
        else:
            side = max(2, int(round(n ** (1.0 / 3.0))))
            a = P.grid_stencil((side, side, side), P.stencil_offsets_3d(pts))
    elif f == "banded":
        a = P.banded(n, spec["half_bw"], spec["fill"], s)
    elif f == "fem3":
        side = max(2, int(round((n / 3.0) ** (1.0 / 3.0))))
        a = P.kuhn_tet(side, side, side, 3)
    else:
        a = P.power_law(n, spec["mean_deg"], spec["exponent"], s)
        order = "random"
    fill_values(a, s, kind)
    if order == "random":
        a = P.reorder(a, P.random_order(a.n, s + 7))
    elif order == "rcm":
        a = P.reorder(a, P.rcm_order(a))
    x = vector(a, s + 100, kind)
    a.meta["name"] = f"fam{spec['m']}_{f}_{a.n}"
    a.meta["spec"] = spec
    return a, x

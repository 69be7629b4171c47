"""Host-side library logic against the oracle (no GPU needed).

csrc_from_csr, csrc_quantize, csrc_color and the plan's tiles must agree with
the oracle bit for bit; plan windows and pull lists must cover every scatter
exactly once.  Also checks that libcsrc exports every symbol csrc.h declares.
"""

import os
import re

import numpy as np
import pytest

from oracle import reference as R
from synth import patterns as P, workloads as W
from synth.values import fill_values

import paper_1003_0952_amd as C
from paper_1003_0952_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "csrc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(csrc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared_symbols()
    assert len(names) >= 30
    for name in names:
        assert hasattr(B.lib, name), name
    assert B.lib.csrc_version() >= 10000


MATS = [
    lambda: W.quad64()[0],
    lambda: W.hex_mesh(11)[0],
    lambda: W.hex_mesh(11, "random")[0],
    lambda: W.hex_mesh(11, "rcm")[0],
    lambda: W.tet_mesh(5)[0],
    lambda: fill_values(P.banded(2500, 40, 0.25, 3), 4),
    lambda: fill_values(P.reorder(P.power_law(4000, 16.0, 2.5, 7), P.random_order(4000, 8)), 5),
]


@pytest.mark.parametrize("make", MATS)
def test_from_csr_bit_exact(make):
    a = make()
    ref = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    got = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    assert got["k"] == ref["k"]
    for key in ("ia", "ja"):
        assert np.array_equal(got[key], ref[key]), key
    for key in ("ad", "al", "au"):
        assert np.array_equal(got[key].view(np.uint64), ref[key].view(np.uint64)), key


def test_from_csr_unsorted_and_errors():
    a = W.hex_mesh(5)[0]
    rng = np.random.default_rng(1)
    col, val = a.col.copy(), a.val.copy()
    for i in range(a.n):
        s, e = a.rowptr[i], a.rowptr[i + 1]
        p = rng.permutation(e - s) + s
        col[s:e], val[s:e] = a.col[p], a.val[p]
    ref = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    got = C.csrc_from_csr(a.n, a.rowptr, col, val)
    for key in ("ia", "ja", "ad", "al", "au"):
        assert np.array_equal(got[key], ref[key])
    cases = [
        ((2, [0, 2, 3], [0, 0, 1], [1.0, 1.0, 1.0]), B.ERR_DUPLICATE),
        ((2, [0, 1, 2], [0, 2], [1.0, 1.0]), B.ERR_INDEX_RANGE),
        ((2, [0, 1, 3], [0, 0, 1], [1.0, 1.0, 1.0]), B.ERR_NOT_STRUCT_SYM),
        ((2, [0, 1, 3], [0, 0, -1], [1.0, 1.0, 1.0]), B.ERR_INDEX_RANGE),
    ]
    for args, code in cases:
        with pytest.raises(C.CsrcError) as e:
            C.csrc_from_csr(*args)
        assert e.value.status == code
    got = C.csrc_from_csr(2, [0, 1, 3], [0, 0, 1], [1.0, 7.0, 2.0], pad=True)
    ref = R.csr_to_csrc(2, [0, 1, 3], [0, 0, 1], [1.0, 7.0, 2.0], pad=True)
    for key in ("ia", "ja", "ad", "al", "au"):
        assert np.array_equal(got[key], ref[key])
    z = C.csrc_from_csr(0, [0], [], [])
    assert z["k"] == 0


def test_quantize_bit_exact():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.uniform(-3, 3, 10000), [0.0, -0.0, 1 + 2**-8, 1 + 3 * 2**-9, 1e-40, 3e38,
                                                    np.inf, -np.inf]])
    assert np.array_equal(C.csrc_quantize(v, "f32").view(np.uint32), R.to_f32(v).view(np.uint32))
    assert np.array_equal(C.csrc_quantize(v, "bf16"), R.to_bf16_bits(v))
    assert np.array_equal(C.csrc_quantize(v, "f64"), v)


COLOR_MATS = [
    lambda: W.quad64()[0],
    lambda: P.q1_hex(16, 16, 16),
    lambda: P.reorder(P.q1_hex(9, 9, 9), P.random_order(729, 2)),
    lambda: P.kuhn_tet(6, 6, 6, 3),
    lambda: P.banded(3000, 20, 0.3, 2),
    lambda: P.power_law(3000, 12.0, 2.5, 4),
]


@pytest.mark.parametrize("make", COLOR_MATS)
@pytest.mark.parametrize("criterion", [0, 1])
def test_colouring_bit_exact(make, criterion):
    a = make()
    if a.val is None:
        fill_values(a, 1)
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    ref, nref = R.color(c, criterion)
    got, ngot = C.csrc_color(c["ia"], c["ja"], criterion)
    assert ngot == nref
    assert np.array_equal(got, ref)


def host_matrix(a):
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)

    class H:
        pass
    h = H()
    h.n, h.k, h.vdtype = c["n"], c["k"], 0
    h.host_ia, h.host_ja, h.device = c["ia"], c["ja"], "cpu"
    return c, h


class HostPlan(C.Plan):
    """Plan built on the host only (no workspace upload)."""

    def __init__(self, h, variant, **kw):
        import ctypes
        opts = B.PlanOpts()
        B.check(B.lib.csrc_plan_opts_default(B.VARIANTS[variant], ctypes.byref(opts)))
        for k, v in kw.items():
            setattr(opts, k, v)
        hh = ctypes.c_void_p(0)
        B.check(B.lib.csrc_plan_create(h.n, B.np_ptr(h.host_ia), B.np_ptr(h.host_ja), 0,
                                       ctypes.byref(opts), ctypes.byref(hh)))
        self._h = hh


@pytest.mark.parametrize("make", MATS[:5])
@pytest.mark.parametrize("work", [512, 4096, 30000])
def test_plan_tiles_match_partition(make, work):
    c, h = host_matrix(make())
    # row caps: a tile keeps per-row state in LDS (2048 rows); an owner tile
    # also serves products with strided or several right-hand sides, whose
    # sums take rows x 5 FP64 values (a group of 4 lanes) within 36 KiB
    for variant, cap in (("atomic", 2048), ("private", 2048), ("owner", 921)):
        p = HostPlan(h, variant, tile_work=work)
        assert np.array_equal(p.export(0), R.partition_for_target(c["ia"], work, cap))


@pytest.mark.parametrize("make", MATS[:5])
def test_private_windows_cover_effective_ranges(make):
    c, h = host_matrix(make())
    p = HostPlan(h, "private", tile_work=2048)
    tiles = p.export(0)
    iv = p.export(2).reshape(-1, 3)
    for t in range(len(tiles) - 1):
        r0, r1 = tiles[t], tiles[t + 1]
        mine = iv[iv[:, 0] == t]
        need = R.out_of_tile_targets(c, r0, r1)
        covered = np.concatenate([np.arange(s, s + L) for _, s, L in mine]) if len(mine) else np.zeros(0, int)
        # intervals are disjoint, ascending, below r0, and contain every target
        assert np.all(np.diff(covered) > 0)
        assert covered.size == 0 or covered.max() < r0
        assert np.all(np.isin(need, covered))
    info = p.info()
    assert info["window_slots"] == sum(iv[:, 2])


@pytest.mark.parametrize("make", MATS[:5])
def test_owner_pull_lists_cover_every_scatter(make):
    c, h = host_matrix(make())
    p = HostPlan(h, "owner", tile_work=2048)
    tiles = p.export(0)
    iv = p.export(2).reshape(-1, 3)
    tile_of = np.searchsorted(tiles, np.arange(c["n"]), side="right") - 1
    rows = np.repeat(np.arange(c["n"]), np.diff(c["ia"]))
    ti, tj = tile_of[rows], tile_of[c["ja"]]
    cross = ti != tj
    pulled = set()
    for t, s, L in iv:
        for r in range(s, s + L):
            pulled.add((t, r))
    for r, t in zip(rows[cross], tj[cross]):
        assert (t, r) in pulled


def test_plan_options_rejected():
    c, h = host_matrix(W.quad64()[0])
    with pytest.raises(C.CsrcError):
        HostPlan(h, "private", lanes=3)
    with pytest.raises(C.CsrcError):
        HostPlan(h, "private", block=100)
    # atomic merge: PRIVATE only, not compensated
    for variant, kw in (("atomic", {}), ("owner", {}), ("private", {"compensated": 1}),
                        ("private", {"atomic_merge": 2})):
        kw = dict(kw)
        kw.setdefault("atomic_merge", 1)
        with pytest.raises(C.CsrcError) as e:
            HostPlan(h, variant, **kw)
        assert e.value.status == -1, (variant, kw)
    # the reserved fields must be zero
    for kw in ({"persistent": 1}, {"grid": 16}):
        with pytest.raises(C.CsrcError) as e:
            HostPlan(h, "private", **kw)
        assert e.value.status == -1, kw


def test_features_definition():
    a, _ = W.quad64()
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    f = C.csrc_features(c["ia"], c["ja"], "f64", -1)
    lens = np.diff(a.rowptr)
    assert f[0] == pytest.approx(np.log2(a.n + 1))
    assert f[1] == pytest.approx(np.log2(a.nnz + 1))
    assert f[2] == pytest.approx(lens.mean(), rel=1e-6)
    assert f[3] == pytest.approx(lens.var(), rel=1e-5)
    assert f[5] == pytest.approx(65 / 4096)
    assert f[9] == pytest.approx(7 / 32)
    assert f[11] == 0.0
    t = P.kuhn_tet(4, 4, 4, 3)
    fill_values(t, 1)
    ct = R.csr_to_csrc(t.n, t.rowptr, t.col, t.val)
    assert C.csrc_features(ct["ia"], ct["ja"], "f64", 3)[11] == 1.0


def test_features_oracle_hand_values():
    # 1D Laplacian pattern on 6 rows: lower pairs (i, i-1); lengths 2,3,3,3,3,2
    from oracle import features as OF
    n = 6
    rows = [i for i in range(n) for _ in (0,)] + list(range(1, n)) + list(range(0, n - 1))
    cols = list(range(n)) + list(range(0, n - 1)) + list(range(1, n))
    key = np.unique(np.array(rows) * n + np.array(cols))
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(key // n, minlength=n), out=rp[1:])
    c = R.csr_to_csrc(n, rp, key % n, np.ones(key.size))
    f = OF.features(c)
    assert f[0] == np.log2(7) and f[1] == np.log2(17)
    assert f[2] == pytest.approx(16 / 6) and f[4] == pytest.approx(3 / (16 / 6))
    assert f[5] == pytest.approx(1 / 6) and f[6] == pytest.approx(1 / 6) and f[7] == 1.0
    assert f[8] == np.log2(3.0) and f[9] == 2 / 32 and f[11] == 0.0


@pytest.mark.parametrize("make", MATS)
def test_features_match_oracle(make):
    from oracle import features as OF
    a = make()
    c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    got = C.csrc_features(c["ia"], c["ja"], "f64", -1)
    assert np.allclose(got, OF.features(c), rtol=2e-6, atol=1e-6)


@pytest.mark.parametrize("side", [3, 6])
def test_rect_split_bit_exact(side):
    """The library's A_S / A_R split (Sec. 2.1) equals the oracle's."""
    (n, m, rowptr, col, val), _ = W.rect_mesh(side)
    (srp, scol, sval), r = C.csrc_rect_split(n, m, rowptr, col, val)
    (orp, ocol, oval), o = R.split_rect(n, m, rowptr, col, val)
    assert np.array_equal(srp, orp) and np.array_equal(scol, ocol) and np.array_equal(sval, oval)
    for key in ("iar", "jar", "ar"):
        assert np.array_equal(r[key], o[key]), key
    assert r["kr"] == o["kr"] and r["m"] == m


def test_rect_split_rejects_bad_columns():
    rowptr = np.array([0, 2, 3], np.int64)
    col = np.array([0, 5, 1], np.int32)
    with pytest.raises(C.CsrcError) as e:
        C.csrc_rect_split(2, 4, rowptr, col, np.ones(3))
    assert e.value.status == B.ERR_INDEX_RANGE
    with pytest.raises(C.CsrcError):
        C.csrc_rect_split(3, 2, np.zeros(4, np.int64), np.zeros(0, np.int32), np.zeros(0))   # m < n


@pytest.mark.parametrize("make", MATS[:5])
@pytest.mark.parametrize("work", [1024, 4096])
def test_tile_colour_classes(make, work):
    """TILE_COLOR plan: tiles as PRIVATE's, window intervals covering each
    tile's effective range (Sec. 3.1), and tile colours equal to the oracle's
    greedy first-fit over the rows each tile writes (bit-exact)."""
    c, h = host_matrix(make())
    p = HostPlan(h, "tile_color", tile_work=work)
    tiles = p.export(0)
    assert np.array_equal(tiles, R.partition_for_target(c["ia"], work, 2048))
    iv = p.export(2).reshape(-1, 3)
    sets = []
    for t in range(len(tiles) - 1):
        r0, r1 = tiles[t], tiles[t + 1]
        mine = iv[iv[:, 0] == t]
        win = np.concatenate([np.arange(s, s + L) for _, s, L in mine]) if len(mine) else np.zeros(0, int)
        assert np.all(np.isin(R.out_of_tile_targets(c, r0, r1), win))
        sets.append(np.concatenate([np.arange(r0, r1), win]))
    col = p.export(1)
    ref, nref = R.color_blocks(sets)
    assert np.array_equal(col, ref)
    assert p.info()["ncolors"] == nref


def test_tile_colour_options_rejected():
    c, h = host_matrix(W.quad64()[0])
    with pytest.raises(C.CsrcError):
        HostPlan(h, "tile_color", max_rhs=4)

"""Pins for the oracle's colouring (Sec. 3.2) and nnz-guided partition (Sec. 3.1).

The colouring is checked by brute force: validity (no two rows of a colour
conflict) and the first-fit property (each colour below a row's colour is
taken by an earlier conflicting row), which together fix greedy first-fit in
ascending row order uniquely; plus closed forms on special patterns.
"""

import numpy as np
import pytest

from oracle import reference as R
from synth import patterns as P, workloads as W
from synth.values import fill_values


def csrc_of(a):
    if a.val is None:
        fill_values(a, 1)
    return R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)


def brute_force_check(c, color, criterion):
    conf = R.conflicts_py(c, criterion)
    for i in range(c["n"]):
        for r in conf[i]:
            assert color[r] != color[i], (i, r)
        earlier = {color[r] for r in conf[i] if r < i}
        for k in range(color[i]):
            assert k in earlier, (i, k)


SMALL = [
    lambda: P.q1_quad(9, 7),
    lambda: P.q1_hex(4, 4, 3),
    lambda: P.reorder(P.q1_hex(4, 4, 4), P.random_order(64, 3)),
    lambda: P.kuhn_tet(3, 3, 3, 3),
    lambda: P.banded(120, 9, 0.4, 2),
    lambda: P.power_law(200, 8.0, 2.5, 9),
]


@pytest.mark.parametrize("make", SMALL)
@pytest.mark.parametrize("criterion", [R.WRITE_SET, R.DISTANCE2])
def test_colouring_brute_force(make, criterion):
    c = csrc_of(make())
    col, nc = R.color(c, criterion)
    brute_force_check(c, col, criterion)
    assert nc == col.max() + 1
    col2, nc2 = R.color_py(c, criterion)
    assert np.array_equal(col, col2) and nc == nc2


def test_colouring_closed_forms():
    n = 30
    tri = P.banded(n, 1, 1.0, 0)
    c = csrc_of(tri)
    col, nc = R.color(c, R.WRITE_SET)
    assert np.array_equal(col, np.arange(n) % 2) and nc == 2
    col, nc = R.color(c, R.DISTANCE2)
    assert np.array_equal(col, np.arange(n) % 3) and nc == 3
    diag = P.banded(n, 0, 1.0, 0)
    c = csrc_of(diag)
    assert R.color(c, R.WRITE_SET)[1] == 1
    full = P.banded(n, n - 1, 1.0, 0)
    c = csrc_of(full)
    col, nc = R.color(c, R.WRITE_SET)
    assert nc == n and np.array_equal(col, np.arange(n))


def test_colouring_lower_bound_and_sizes():
    # every y entry t is written by {t} and by all rows storing t as a lower
    # column; those writers pairwise conflict, so C >= max writers.
    for a, crit_counts in ((P.q1_quad(64, 64), (7, 9)), (P.q1_hex(16, 16, 16), (24, 27))):
        c = csrc_of(a)
        writers = 1 + np.bincount(c["ja"], minlength=c["n"])
        for crit, expect in zip((R.WRITE_SET, R.DISTANCE2), crit_counts):
            col, nc = R.color(c, crit)
            assert nc >= writers.max()
            assert nc == expect
            # large-n validity: each y index written by at most one row per colour
            rows = np.repeat(np.arange(c["n"]), np.diff(c["ia"]))
            tgt = np.concatenate([np.arange(c["n"]), c["ja"]])
            who = np.concatenate([np.arange(c["n"]), rows])
            key = tgt.astype(np.int64) * nc + col[who]
            assert np.unique(key).shape[0] == key.shape[0]


def test_partition_definition():
    for a in (P.q1_hex(10, 10, 10), P.power_law(3000, 30.0, 2.5, 2), P.banded(500, 3, 0.5, 1)):
        c = csrc_of(a)
        w = R.row_weights(c["ia"])
        C = np.concatenate([[0], np.cumsum(w)])
        total = C[-1]
        for parts in (1, 2, 3, 7, 64, 1000):
            s = R.partition(c["ia"], parts)
            assert s[0] == 0 and s[-1] == c["n"] and np.all(np.diff(s) >= 0)
            for b in range(1, parts):
                i = s[b]
                assert C[i] * parts >= b * total
                assert i == 0 or C[i - 1] * parts < b * total
            # balance: no block exceeds the average by more than one row
            blocks = C[s[1:]] - C[s[:-1]]
            assert blocks.max() <= total / parts + w.max()


def test_partition_weights_are_nnz():
    a = P.q1_hex(6, 6, 6)
    c = csrc_of(a)
    assert R.row_weights(c["ia"]).sum() == a.nnz


def test_drop_empty_blocks():
    """Tiles are the non-empty blocks: repeated boundaries go, the covered
    rows and every non-empty block stay."""
    assert list(R.drop_empty([0, 0, 3, 3, 3, 7, 9, 9])) == [0, 3, 7, 9]
    assert list(R.drop_empty([0, 5])) == [0, 5]
    c = csrc_of(P.banded(300, 40, 1.0, 3))
    total = int(R.row_weights(c["ia"]).sum())
    for target in (1, 10, 81, 500):
        s = R.partition(c["ia"], max(1, -(-total // target)))
        t = R.partition_for_target(c["ia"], target)
        assert t[0] == 0 and t[-1] == c["n"] and np.all(np.diff(t) > 0)
        assert set(t.tolist()) == set(R.cap_rows(s, 2048).tolist())
    # one row per tile when the target is below every row's work
    assert list(R.partition_for_target(c["ia"], 1)) == list(range(301))


def test_out_of_tile_targets_brute_force():
    c = csrc_of(P.q1_hex(7, 7, 7))
    s = R.partition(c["ia"], 9)
    for b in range(9):
        r0, r1 = s[b], s[b + 1]
        expect = set()
        for i in range(r0, r1):
            for q in range(c["ia"][i], c["ia"][i + 1]):
                if c["ja"][q] < r0:
                    expect.add(int(c["ja"][q]))
        assert list(R.out_of_tile_targets(c, r0, r1)) == sorted(expect)


def test_row_cap():
    bounds = np.array([0, 5, 5, 4100, 4200, 10000])
    capped = R.cap_rows(bounds, 2048)
    # 4095 rows -> 2 pieces, 5800 rows -> 3 pieces, the rest unchanged
    assert list(capped) == [0, 5, 5, 5 + 4095 // 2, 4100, 4200, 4200 + 5800 // 3,
                            4200 + 2 * 5800 // 3, 10000]
    assert np.all(np.diff(capped) <= 2048) and np.all(np.diff(capped) >= 0)


def _block_brute_force(sets, col):
    """Validity and the first-fit property of a block colouring."""
    S = [set(int(r) for r in w) for w in sets]
    for b in range(len(S)):
        for d in range(len(S)):
            if d != b and S[b] & S[d]:
                assert col[b] != col[d], (b, d)
        earlier = {col[d] for d in range(b) if S[b] & S[d]}
        for k in range(col[b]):
            assert k in earlier, (b, k)


def test_block_colouring_brute_force():
    rng = np.random.default_rng(7)
    for trial in range(20):
        nb = int(rng.integers(1, 40))
        sets = [rng.choice(60, size=int(rng.integers(0, 6)), replace=False) for _ in range(nb)]
        col, nc = R.color_blocks(sets)
        _block_brute_force(sets, col)
        assert nc == (col.max() + 1 if nb else 0)


def test_block_colouring_closed_forms():
    # disjoint sets: one class; a chain where only neighbours overlap: two
    # alternating classes; one shared row: every block its own class
    col, nc = R.color_blocks([[3 * b, 3 * b + 1] for b in range(10)])
    assert nc == 1 and not col.any()
    col, nc = R.color_blocks([[b, b + 1] for b in range(10)])
    assert nc == 2 and np.array_equal(col, np.arange(10) % 2)
    col, nc = R.color_blocks([[5, 100 + b] for b in range(7)])
    assert nc == 7 and np.array_equal(col, np.arange(7))
    assert R.color_blocks([])[1] == 0


@pytest.mark.parametrize("make", SMALL[:4])
def test_block_colouring_of_single_rows_is_row_colouring(make):
    """With one row per block and its write set W(i), the block colouring is
    the greedy row colouring of Sec. 3.2 (pinned above by brute force)."""
    c = csrc_of(make())
    sets = [R.write_set(c, i) for i in range(c["n"])]
    col, nc = R.color_blocks(sets)
    ref, nref = R.color(c, R.WRITE_SET)
    assert np.array_equal(col, ref) and nc == nref

"""The exhaustive autotuner: its candidate list and timing database (host
logic), and on the GPU a full tuning pass whose pick is the fastest candidate
and computes the product the oracle computes."""

import numpy as np
import pytest

from oracle import reference as R
from synth import workloads as W
from tests.helpers import oracle_csrc, rel_inf

from paper_1003_0952_amd import tuner as T


def test_candidate_names_unique_and_defaults_in_range():
    names = [T.candidate_name(i) for i in range(len(T.CANDIDATES))]
    assert len(set(names)) == len(names)
    for i in (T.DEFAULT, T.FALLBACK, T.PLAIN):
        assert 0 <= i < len(T.CANDIDATES)
    assert T.CANDIDATES[T.PLAIN][0] == "plain"
    assert len({tuple(sorted(c.items())) for c in T.BATCH_CANDIDATES}) == len(T.BATCH_CANDIDATES)


def test_timing_db_resumes(tmp_path):
    path = str(tmp_path / "db.jsonl")
    db = T.TimingDB(path)
    assert db.get("k", "c") is None
    db.put("k", "c", 12.5, extra=1)
    db.put("k", "d", float("inf"))
    db.put("k", "c", 11.0)          # a later record replaces the earlier one
    again = T.TimingDB(path)
    assert again.get("k", "c") == 11.0
    assert again.get("k", "d") == float("inf")
    assert again.get("other", "c") is None


class _Host:
    def __init__(self, a):
        c = oracle_csrc(a)
        self.n, self.host_ia, self.host_ja = c["n"], c["ia"], c["ja"]


def test_structure_hash_tracks_pattern_only():
    a, _ = W.quad64(side=16)
    b, _ = W.quad64(kind="int", side=16)   # same pattern, other values
    c, _ = W.quad64(side=17)
    assert T.structure_hash(_Host(a)) == T.structure_hash(_Host(b))
    assert T.structure_hash(_Host(a)) != T.structure_hash(_Host(c))


@pytest.mark.gpu
def test_tune_picks_fastest_and_pick_is_correct(tmp_path):
    import torch
    import paper_1003_0952_amd as C
    a, x = W.hex_mesh(12, "natural")
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    mats = [C.Matrix(host, "f64") for _ in range(2)]
    xs = [torch.from_numpy(x).cuda() for _ in range(2)]
    ys = [torch.empty(a.n, dtype=torch.float64, device="cuda") for _ in range(2)]
    db = T.TimingDB(str(tmp_path / "t.jsonl"))
    key = T.structure_hash(mats[0])
    times, best = T.tune(torch, mats, xs, ys, db=db, key=key, warmup=1, reps=2, runs=1)
    assert len(times) == len(T.CANDIDATES)
    assert best == int(np.argmin(times)) and np.isfinite(times[best])
    assert all(t > 0 for t in times)
    # a second pass is served from the database
    times2, best2 = T.tune(torch, mats, xs, ys, db=T.TimingDB(str(tmp_path / "t.jsonl")), key=key)
    assert times2 == times and best2 == best
    v, kw = T.CANDIDATES[best]
    plan = C.Plan(mats[0], v, **kw)
    c = oracle_csrc(a)
    for tr in (False, True):
        y = (C.csrc_spmv_t if tr else C.csrc_spmv)(mats[0], plan, xs[0], ys[0])
        torch.cuda.synchronize()
        assert rel_inf(y.cpu().numpy(), (R.spmv_t if tr else R.spmv)(c, x)) <= 1e-12

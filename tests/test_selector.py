"""The trained selector on its stored campaign (timings measured on MI355X by
paper_1003_0952_amd.train_selector in FP64, FP32 and BF16 storage, on the
current kernel sources; network trained on the GPU): what the network gains
over the fixed choice without it, on held-out matrices."""

import json
import os

import numpy as np
import pytest

from paper_1003_0952_amd import selector as S, tuner as T
from paper_1003_0952_amd.train_selector import load_db, samples, evaluate, heldout_ranges, is_heldout

DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1003_0952_amd",
                    "selector_data")


@pytest.fixture(scope="module")
def stored():
    from paper_1003_0952_amd.sources import kernel_source_hash
    recs, stale = load_db(os.path.join(DATA, "timings.jsonl"), kernel_source_hash("single"))
    model = S.Selector.load(os.path.join(DATA, "model.json"))
    assert model is not None and model.K == len(T.CANDIDATES)
    return recs, model


COUNT = 2240          # 2000 matrices up to 2e6 nnz, then 240 up to 3e7 nnz
BIG_FROM = 2000
HELDOUT = heldout_ranges("1800:2000,2200:2240")
DTYPES = ("f64", "f32", "bf16")
GAIN_MIN = 1.08       # geometric-mean speedup over the fixed choice, held out
REGRET_MAX = 0.06     # mean regret against exhaustive tuning, held out, per storage type


def heldout(recs):
    return samples([r for r in recs if is_heldout(r["m"], HELDOUT)])


def test_campaign_shape(stored):
    """Every matrix of the family timed in every storage type on the current
    kernel sources."""
    recs, _ = stored
    assert len(recs) == COUNT
    assert {r["m"] for r in recs} == set(range(COUNT))
    assert max(r["nnz"] for r in recs if r["m"] >= BIG_FROM) > 2e6
    fams = {r["spec"]["family"] for r in recs}
    assert fams == {"stencil", "banded", "fem3", "power"}
    for r in recs:
        assert set(r["dtypes"]) == set(DTYPES)
        for d in r["dtypes"].values():
            assert len(d["features"]) == 12 and len(d["times_us"]) == len(T.CANDIDATES)
            assert d["best"] == int(np.argmin(d["times_us"]))


def test_stale_records_are_refused(tmp_path):
    """Records taken on other kernel sources are skipped (and counted)."""
    from paper_1003_0952_amd.sources import kernel_source_hash
    src = kernel_source_hash("single")
    rec = {"m": 0, "spec": {}, "n": 1, "nnz": 1, "candidates": [],
           "dtypes": {"f64": {"features": [0.0] * 12, "times_us": [1.0], "best": 0}}}
    path = tmp_path / "t.jsonl"
    with open(path, "w") as fh:
        fh.write(json.dumps(dict(rec, src="0" * 16)) + "\n")
        fh.write(json.dumps(dict(rec, m=1, src=src)) + "\n")
        fh.write(json.dumps(dict(rec, m=2)) + "\n")                 # no hash at all
    recs, stale = load_db(str(path), src)
    assert [r["m"] for r in recs] == [1] and stale == 2


def test_heldout_gain_over_fixed_choice(stored):
    recs, model = stored
    held = heldout(recs)
    assert len(held) == 240 * len(DTYPES)
    ev = evaluate(model, held, T.DEFAULT, T.FALLBACK)
    assert ev["gain_vs_default_geomean"] > GAIN_MIN     # faster than the fixed choice
    assert ev["regret_mean"] < REGRET_MAX               # close to exhaustive tuning
    assert ev["exact_pick_rate"] > 0.6
    for dt in DTYPES:
        e = evaluate(model, [h for h in held if h["dtype"] == dt], T.DEFAULT, T.FALLBACK)
        assert e["regret_mean"] < REGRET_MAX, dt
    # a pick the library cannot plan for a matrix is rare; the caller then
    # takes the fixed choice (evaluate and selector.choose both do)
    bad = [h for h in held if not np.isfinite(h["times_us"][model.predict(np.array(h["features"], np.float32))])]
    assert len(bad) <= len(held) // 100


def test_report_matches_stored_data(stored):
    from paper_1003_0952_amd.sources import kernel_source_hash
    recs, model = stored
    with open(os.path.join(DATA, "report.json")) as fh:
        rep = json.load(fh)
    assert rep["kernel_source_hash"] == kernel_source_hash("single")
    held = heldout(recs)
    ev = evaluate(model, held, T.DEFAULT, T.FALLBACK)
    assert rep["heldout_samples"] == len(held)
    assert rep["heldout"]["exact_pick_rate"] == pytest.approx(ev["exact_pick_rate"])
    assert rep["heldout"]["gain_vs_default_geomean"] == pytest.approx(ev["gain_vs_default_geomean"])


@pytest.mark.parametrize("m", [1800, 1803, 1950, 2201])
def test_stored_features_are_the_library_features(stored, m):
    from synth import workloads as W
    import paper_1003_0952_amd as C
    recs, _ = stored
    rec = next(r for r in recs if r["m"] == m)
    spec = W.family_spec(m, nnz_cap=3e7 if m >= BIG_FROM else 2e6)
    assert spec == rec["spec"]
    a, _ = W.family_member(spec)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    for dt in DTYPES:
        f = C.csrc_features(host["ia"], host["ja"], dt, -1)
        assert np.allclose(f, rec["dtypes"][dt]["features"], rtol=1e-6), dt


def test_csrc_select_matches_features_then_network(stored):
    """csrc_select (library features + host network) picks the same class as
    the two steps called one by one, and reports a missing model so the
    caller can tune instead."""
    import ctypes
    from paper_1003_0952_amd import api as C, binding as B
    from synth import workloads as W
    _, model = stored
    for a, _x in (W.quad64(), W.hex_mesh(17, "natural"), W.hex_mesh(17, "random"), W.tet_mesh(6)):
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        want = model.predict(C.csrc_features(host["ia"], host["ja"], "f64"))
        assert model.select(host["n"], host["ia"], host["ja"]) == want
    ia = np.ascontiguousarray(host["ia"], np.int32)
    ja = np.ascontiguousarray(host["ja"], np.int32)
    c = ctypes.c_int32(-5)
    st = B.lib.csrc_select(host["n"], B.np_ptr(ia), B.np_ptr(ja), B.F64, model.H, model.K, None, None, None,
                           ctypes.byref(c))
    assert st == B.ERR_NO_MODEL and c.value == -5
    assert b"model" in B.lib.csrc_status_string(st)


@pytest.mark.parametrize("hidden,classes", [(0, 10), (64, 65), (257, 10), (64, 0)])
def test_csrc_select_rejects_bad_network_shape(hidden, classes):
    """A network shape outside the library's limits is an argument error
    (checked before the features, which colour the rows), and *candidate
    stays untouched."""
    import ctypes
    from paper_1003_0952_amd import api as C, binding as B
    from synth import workloads as W
    a, _ = W.hex_mesh(12, "natural")
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    ia = np.ascontiguousarray(host["ia"], np.int32)
    ja = np.ascontiguousarray(host["ja"], np.int32)
    params = np.zeros(70000, np.float32)
    mean = np.zeros(12, np.float32)
    scale = np.ones(12, np.float32)
    c = ctypes.c_int32(-5)
    st = B.lib.csrc_select(host["n"], B.np_ptr(ia), B.np_ptr(ja), B.F64, hidden, classes, B.np_ptr(params),
                           B.np_ptr(mean), B.np_ptr(scale), ctypes.byref(c))
    assert st == B.ERR_ARG and c.value == -5
    # the same call with a valid shape picks a class
    st = B.lib.csrc_select(host["n"], B.np_ptr(ia), B.np_ptr(ja), B.F64, 64, 10, B.np_ptr(params),
                           B.np_ptr(mean), B.np_ptr(scale), ctypes.byref(c))
    assert st == B.OK and 0 <= c.value < 10

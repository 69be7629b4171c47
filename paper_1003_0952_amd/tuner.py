"""Exhaustive autotuner: time every candidate (variant x tile shape) on a
matrix and keep the fastest.  It is the learned selector's fallback and the
yardstick of its regret.

Timing protocol: HIP events on the current stream around `reps` products
after `warmup` products; the median of `runs` such means.  Matrices larger
than a third of the 256 MiB Infinity Cache are timed over rotated copies
passed in by the caller.  Results go to a resumable JSON-lines database
keyed by (structure hash, value type, candidate).
"""

import hashlib
import json
import os

import numpy as np

from . import api as C

# (variant, plan options).  Order fixes the class index of the selector.
CANDIDATES = [
    ("private", {"tile_work": 4096, "block": 256}),
    ("private", {"tile_work": 8192, "block": 256}),
    ("private", {"tile_work": 16384, "block": 512}),
    ("private", {"tile_work": 4096, "block": 256, "atomic_merge": 1}),
    ("private", {"tile_work": 8192, "block": 256, "atomic_merge": 1}),
    ("private", {"tile_work": 16384, "block": 512, "atomic_merge": 1}),
    ("owner", {"tile_work": 8192, "block": 512}),
    ("atomic", {"tile_work": 8192, "block": 512}),
    ("color", {}),
    ("plain", {}),
]
DEFAULT = 1      # the fixed choice without a selector: private, 8192, 256 threads, merge pass
FALLBACK = 7     # ... or atomic, 8192, 512 threads where private cannot run
PLAIN = 9        # ... or the plain kernel, which runs every matrix

# Batched products (one persistent launch over many matrices): tile form,
# work item size and threads per workgroup, timed on the whole batch.
BATCH_CANDIDATES = [
    {"variant": "owner", "tile_work": 4096, "block": 512},
    {"variant": "owner", "tile_work": 16384, "block": 512},
    {"variant": "owner", "tile_work": 32768, "block": 1024},
    {"variant": "private", "tile_work": 16384, "block": 512},
]


def candidate_name(i):
    v, kw = CANDIDATES[i]
    return v + "".join(f"_{k}{kw[k]}" for k in sorted(kw))


def structure_hash(A):
    h = hashlib.sha1()
    h.update(np.int64(A.n).tobytes())
    h.update(A.host_ia.tobytes())
    h.update(A.host_ja.tobytes())
    return h.hexdigest()[:16]


def time_candidate(torch, mats, xs, ys, variant, kw, warmup=2, reps=5, runs=3, transpose=False):
    """Median over `runs` of the mean product time (microseconds); inf if the
    variant cannot run this matrix."""
    try:
        plan = C.Plan(mats[0], variant, **kw)
    except C.CsrcError:
        return float("inf")
    f = C.csrc_spmv_t if transpose else C.csrc_spmv
    nc = len(mats)
    for s in range(warmup):
        f(mats[s % nc], plan, xs[s % nc], ys[s % nc])
    out = []
    for _ in range(runs):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for s in range(reps):
            f(mats[s % nc], plan, xs[s % nc], ys[s % nc])
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) * 1e3 / reps)
    return float(np.median(out))


class TimingDB:
    """Append-only JSON lines: one record per (key, candidate)."""

    def __init__(self, path):
        self.path = path
        self.rec = {}
        if path and os.path.exists(path):
            with open(path) as fh:
                for line in fh:
                    if line.strip():
                        r = json.loads(line)
                        self.rec[(r["key"], r["cand"])] = r

    def get(self, key, cand):
        r = self.rec.get((key, cand))
        return None if r is None else r["us"]

    def put(self, key, cand, us, **extra):
        r = {"key": key, "cand": cand, "us": us, **extra}
        self.rec[(key, cand)] = r
        if self.path:
            with open(self.path, "a") as fh:
                fh.write(json.dumps(r) + "\n")


def tune(torch, mats, xs, ys, db=None, key=None, candidates=None, **timing):
    """Times of every candidate (list, microseconds) and the index of the best."""
    cands = range(len(CANDIDATES)) if candidates is None else candidates
    times = []
    for i in cands:
        name = candidate_name(i)
        us = db.get(key, name) if db is not None and key else None
        if us is None:
            v, kw = CANDIDATES[i]
            us = time_candidate(torch, mats, xs, ys, v, kw, **timing)
            if db is not None and key:
                db.put(key, name, us)
        times.append(us)
    best = int(np.argmin(times))
    return times, best

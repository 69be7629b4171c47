"""Build the learned selector: time every candidate on seeded matrices of the
selector family, train the network on the GPU, evaluate on held-out matrices.

  python -m paper_1003_0952_amd.train_selector campaign --count 2240 --db DB
  python -m paper_1003_0952_amd.train_selector train --db DB

The campaign is resumable (one JSON line per matrix, with the timings of
every storage type in --dtypes and the hash of the kernel sources; matrices
finished on the current sources are skipped) and stops after --budget
seconds so it can run in several pieces.  Training uses only records of the
current kernel sources, one sample per (matrix, storage type).
Matrices m >= --big-from are drawn with the larger nnz cap.  Matrices in the
--heldout ranges are never trained on.
"""

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DATA = os.path.join(HERE, "selector_data")
MALL = 256 * 2**20


def kernel_source_hash():
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_1003_0952_amd.sources import kernel_source_hash as h
    return h("single")


def _prepare(args):
    """Worker: generate matrix m and its host CSRC arrays and features."""
    m, nnz_cap = args
    sys.path.insert(0, os.path.dirname(HERE))
    from synth import workloads as W
    from paper_1003_0952_amd import api as C
    spec = W.family_spec(m, nnz_cap=nnz_cap)
    a, x = W.family_member(spec)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    f = C.csrc_features(host["ia"], host["ja"], "f64", -1)
    return m, spec, host, x, f


def campaign(args):
    done = set()
    src = kernel_source_hash()
    if os.path.exists(args.db):
        with open(args.db) as fh:
            for line in fh:
                if line.strip():
                    r = json.loads(line)
                    if r.get("src") == src:
                        done.add(r["m"])
    todo = [m for m in range(args.count) if m not in done]
    print(f"# campaign: {len(done)} done, {len(todo)} to go", flush=True)
    if not todo:
        return
    # fork the workers before this process touches the GPU
    pool = ProcessPoolExecutor(max_workers=args.workers)
    import torch
    from paper_1003_0952_amd import api as C, tuner as T
    t0 = time.time()
    threads = ThreadPoolExecutor(max_workers=len(T.CANDIDATES))
    from collections import deque
    pending = deque()
    queue = list(todo)

    def refill():
        # a bounded window of prepared matrices (each may be tens of MB)
        while queue and len(pending) < 2 * args.workers:
            m = queue.pop(0)
            cap = args.big_nnz_cap if m >= args.big_from else args.nnz_cap
            pending.append(pool.submit(_prepare, (m, cap)))

    def results():
        refill()
        while pending:
            r = pending.popleft().result()
            refill()
            yield r

    count = 0
    dtypes = [d for d in args.dtypes.split(",") if d]
    src = kernel_source_hash()
    with open(args.db, "a") as out:
        for m, spec, host, x, f in results():
            per = {}
            for dt in dtypes:
                A = C.Matrix(host, dt)
                ncopy = 3 if A.nbytes() > MALL // 3 else 1
                mats = [A] + [C.Matrix(host, dt) for _ in range(ncopy - 1)]
                xs = [torch.from_numpy(x).to("cuda", A.xdtype) for _ in mats]

                def mk(i):
                    v, kw = T.CANDIDATES[i]
                    try:
                        return C.Plan(A, v, **kw)
                    except C.CsrcError:
                        return None
                plans = list(threads.map(mk, range(len(T.CANDIDATES))))
                times = []
                for p in plans:
                    if p is None:
                        times.append(float("inf"))
                        continue
                    ys = [torch.empty(A.n, dtype=p.ytorch, device="cuda") for _ in mats]
                    for s_ in range(2):
                        C.csrc_spmv(mats[s_ % ncopy], p, xs[s_ % ncopy], ys[s_ % ncopy])
                    runs = []
                    for _ in range(3):
                        e0 = torch.cuda.Event(enable_timing=True)
                        e1 = torch.cuda.Event(enable_timing=True)
                        e0.record()
                        for s_ in range(args.reps):
                            C.csrc_spmv(mats[s_ % ncopy], p, xs[s_ % ncopy], ys[s_ % ncopy])
                        e1.record()
                        torch.cuda.synchronize()
                        runs.append(e0.elapsed_time(e1) * 1e3 / args.reps)
                    times.append(float(np.median(runs)))
                # features of this storage type (the colour count is the FP64 run's)
                feats = f if dt == "f64" else C.csrc_features(host["ia"], host["ja"], dt, int(round(f[9] * 32)))
                per[dt] = {"features": [float(v) for v in feats], "times_us": times,
                           "best": int(np.argmin(times))}
                del plans, mats, xs, A
            rec = {"m": m, "spec": spec, "n": host["n"], "nnz": 2 * host["k"] + host["n"], "src": src,
                   "dtypes": per, "candidates": [T.candidate_name(i) for i in range(len(T.CANDIDATES))]}
            out.write(json.dumps(rec) + "\n")
            out.flush()
            count += 1
            if count % 25 == 0 or (m >= args.big_from and count % 5 == 0):
                print(f"# {count} matrices, {time.time() - t0:.0f}s", flush=True)
            if time.time() - t0 > args.budget:
                print(f"# budget reached after {count} matrices", flush=True)
                queue.clear()
                break
    pool.shutdown(wait=False, cancel_futures=True)
    threads.shutdown(wait=False)
    print(f"# campaign piece done: {count} matrices in {time.time() - t0:.0f}s", flush=True)


def load_db(path, src=None):
    """Records of the current kernel sources (src), one per matrix; records
    taken on other sources are stale and skipped.  Returns (records, stale)."""
    recs, stale = {}, 0
    with open(path) as fh:
        for line in fh:
            if line.strip():
                r = json.loads(line)
                if src is not None and r.get("src") != src:
                    stale += 1
                    continue
                recs[r["m"]] = r
    return [recs[m] for m in sorted(recs)], stale


def samples(recs, dtypes=None):
    """One sample per (matrix, storage type): features, times, best."""
    out = []
    for r in recs:
        for dt, d in r["dtypes"].items():
            if dtypes is None or dt in dtypes:
                out.append({"m": r["m"], "dtype": dt, "features": d["features"], "times_us": d["times_us"],
                            "best": d["best"]})
    return out


def baseline_pick(times, default, fallback):
    """The choice without a selector: the default candidate, else the
    fallback, else the plain kernel (which runs every matrix)."""
    from .tuner import PLAIN
    for c in (default, fallback, PLAIN):
        if np.isfinite(times[c]):
            return c
    return PLAIN


def evaluate(model, recs, default, fallback):
    """Regret of the model's picks against exhaustive tuning, and their gain
    over the fixed choice without a selector, on the given records."""
    ratio, gain, hit, t_model, t_base = [], [], 0, 0.0, 0.0
    for r in recs:
        t = np.array(r["times_us"])
        pick = model.predict(np.array(r["features"], dtype=np.float32))
        tp = t[pick] if np.isfinite(t[pick]) else t[baseline_pick(t, default, fallback)]
        tb = t[baseline_pick(t, default, fallback)]
        ratio.append(tp / t.min())
        gain.append(tb / tp)
        hit += int(pick == int(np.argmin(t)))
        t_model += tp
        t_base += tb
    ratio = np.array(ratio)
    gain = np.array(gain)
    return {"matrices": len(recs), "exact_pick_rate": hit / max(1, len(recs)),
            "regret_mean": float(ratio.mean() - 1), "regret_median": float(np.median(ratio) - 1),
            "regret_geomean": float(np.exp(np.log(ratio).mean()) - 1), "regret_max": float(ratio.max() - 1),
            "gain_vs_default_geomean": float(np.exp(np.log(gain).mean())),
            "gain_vs_default_total_time": float(t_base / t_model)}


def heldout_ranges(text):
    """'1800:2000,2200:2240' -> [(1800, 2000), (2200, 2240)]"""
    return [tuple(int(v) for v in part.split(":")) for part in text.split(",") if part]


def is_heldout(m, ranges):
    return any(a <= m < b for a, b in ranges)


def train_cmd(args):
    import torch
    from paper_1003_0952_amd import selector as S, tuner as T
    recs, stale = load_db(args.db, kernel_source_hash())
    if not recs:
        raise SystemExit(f"no timing records of the current kernel sources ({stale} stale ones)")
    ho = heldout_ranges(args.heldout)
    train_r = samples([r for r in recs if not is_heldout(r["m"], ho)])
    test_r = samples([r for r in recs if is_heldout(r["m"], ho)])
    # cost weighting: a sample counts 1 + log2(slowest runnable / fastest)
    # times (at most args.max_weight), so that matrices on which a wrong pick
    # is expensive weigh more; the library's training kernels take a plain
    # batch, so the weight is a repetition count
    def weight(t):
        t = np.array(t)
        f = t[np.isfinite(t)]
        return int(min(args.max_weight, 1 + np.floor(np.log2(f.max() / f.min())))) if args.max_weight > 1 else 1
    reps = [weight(r["times_us"]) for r in train_r]
    F = np.array([r["features"] for r, w in zip(train_r, reps) for _ in range(w)], dtype=np.float32)
    y = np.array([r["best"] for r, w in zip(train_r, reps) for _ in range(w)], dtype=np.int32)
    K = len(T.CANDIDATES)
    t0 = time.time()
    params, mean, scale, hist = S.train(torch, F, y, K, steps=args.steps, lr=args.lr, seed=args.seed)
    model = S.Selector(params, mean, scale)
    big = [r for r in test_r if r["m"] >= args.big_from]
    dts = sorted({t["dtype"] for t in test_r})
    rep = {"kernel_source_hash": kernel_source_hash(), "stale_records_skipped": stale,
           "train_samples": len(train_r), "heldout_samples": len(test_r), "heldout_ranges": args.heldout,
           "samples": "one per (matrix, storage type); features of csrc_features for that storage type",
           "training_rows": int(len(y)), "max_weight": args.max_weight,
           "steps": args.steps, "seed": args.seed,
           "train_seconds": round(time.time() - t0, 2), "loss_first": hist[0], "loss_last": hist[-1],
           "label_histogram": np.bincount([r["best"] for r in train_r], minlength=K).tolist(),
           "candidates": [T.candidate_name(i) for i in range(K)], "default": T.candidate_name(T.DEFAULT),
           "fallback": T.candidate_name(T.FALLBACK),
           "train": evaluate(model, train_r, T.DEFAULT, T.FALLBACK),
           "heldout": evaluate(model, test_r, T.DEFAULT, T.FALLBACK),
           "heldout_large": evaluate(model, big, T.DEFAULT, T.FALLBACK) if big else None,
           "heldout_by_dtype": {dt: evaluate(model, [t for t in test_r if t["dtype"] == dt], T.DEFAULT, T.FALLBACK)
                                for dt in dts}}
    os.makedirs(os.path.dirname(args.model), exist_ok=True)
    model.save(args.model)
    with open(args.report, "w") as fh:
        json.dump(rep, fh, indent=1)
    print(json.dumps(rep["heldout"]), flush=True)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("campaign")
    c.add_argument("--count", type=int, default=2240)
    c.add_argument("--big-from", type=int, default=2000)
    c.add_argument("--big-nnz-cap", type=float, default=3e7)
    c.add_argument("--db", default=os.path.join(DATA, "timings.jsonl"))
    c.add_argument("--nnz-cap", type=float, default=2e6)
    c.add_argument("--workers", type=int, default=10)
    c.add_argument("--reps", type=int, default=5)
    c.add_argument("--budget", type=float, default=480)
    c.add_argument("--dtypes", default="f64,f32,bf16")
    t = sub.add_parser("train")
    t.add_argument("--db", default=os.path.join(DATA, "timings.jsonl"))
    t.add_argument("--model", default=os.path.join(DATA, "model.json"))
    t.add_argument("--report", default=os.path.join(DATA, "report.json"))
    t.add_argument("--heldout", default="1800:2000,2200:2240")
    t.add_argument("--big-from", type=int, default=2000)
    t.add_argument("--steps", type=int, default=3000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--max-weight", type=int, default=6)
    args = ap.parse_args()
    if args.cmd == "campaign":
        campaign(args)
    else:
        train_cmd(args)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()

#!/usr/bin/env python3
"""Benchmark: CSRC SpMV throughput on one MI355X.

A step is one y = A x and one y = A^T x product (the hot path's pass-1
product, race resolution and transpose) on the 27-point hexahedral mesh of
100^3 nodes (n = 1e6, nnz = 26,463,592), FP64, natural numbering.  Inputs are
resident in HBM before timing.  Successive steps rotate over independent
copies of the matrix and vectors (more than three times the 256 MB Infinity
Cache in total) so each product streams its arrays from HBM.

The variant is chosen outside the timed region by the autotuner (every
candidate timed on this matrix); the learned selector's pick for the same
matrix, and its regret against the tuned choice, are reported beside it.  The
plain FP64 kernel (one thread per row, global atomics) is timed the same way
as the baseline.  Prints one JSON line.

Other workloads: hex100_random / hex100_rcm (the same mesh renumbered),
tet80 (3-dof tetrahedral mesh, for the reduced-precision forms), hex100_sym
(numerically symmetric values, one stored value array), rect100 (the mesh
plus overlap couplings, n x m, A_S + A_R) and batch256 (256 matrices of
uneven size with 1..32 right-hand sides each, run as one persistent launch
under a HIP graph).
"""

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CSRC SpMV HBM GB/s (% peak) & GFLOP/s, tuned/learned vs plain FP64 kernel"
HBM_PEAK_GBS = 8000.0
MALL_BYTES = 256 * 2**20


def algorithmic_bytes(n, k, vbytes, xbytes, ybytes, r=1, symmetric=False):
    """Bytes one product must move: every array once (paper's working set);
    numerically symmetric storage holds one value array (Sec. 2.2)."""
    nv = 1 if symmetric else 2
    return 4 * (n + 1) + k * (4 + nv * vbytes) + n * vbytes + r * n * (xbytes + ybytes)


def flops(n, k, r=1):
    """2 nnz - n per right-hand side (n multiplies, nnz - n multiply-adds)."""
    return r * (2 * (2 * k + n) - n)


def build_workload(name):
    from synth import workloads as W
    if name == "hex100":
        return W.hex_mesh(100, "natural")
    if name == "hex100_random":
        return W.hex_mesh(100, "random")
    if name == "hex100_rcm":
        return W.hex_mesh(100, "rcm")
    if name == "hex100_sym":
        return W.hex_mesh(100, "natural", kind="sym")
    if name.startswith("hex"):
        return W.hex_mesh(int(name[3:]), "natural")
    if name == "tet80":
        return W.tet_mesh(80)
    raise SystemExit(f"unknown workload {name}")


class Copies:
    """Independent device copies of (A, x, y, y_t) for cache-cold rotation."""

    def __init__(self, C, torch, host, dtype, ncopy, x, symmetric=False):
        self.mats = [C.Matrix(host, dtype, symmetric=symmetric) for _ in range(ncopy)]
        xd = self.mats[0].xdtype
        self.x = [torch.from_numpy(x).to("cuda", xd) for _ in range(ncopy)]
        self.y = []
        self.yt = []

    def outputs(self, torch, ydt):
        n = self.mats[0].n
        self.y = [torch.empty(n, dtype=ydt, device="cuda") for _ in self.mats]
        self.yt = [torch.empty(n, dtype=ydt, device="cuda") for _ in self.mats]

    @staticmethod
    def first(cp):
        """A view of cp holding only its first copy (no rotation)."""
        one = Copies.__new__(Copies)
        one.mats, one.x, one.y, one.yt = cp.mats[:1], cp.x[:1], cp.y[:1], cp.yt[:1]
        return one


RUNS = 3   # timed runs per measurement; the median is reported (Sec. 4: median of 3 runs)


def time_plan(C, torch, cp, plan, steps, warmup, runs=RUNS):
    """Milliseconds per step (y = A x, then y = A^T x) of `runs` timed runs
    of `steps` back-to-back steps each, after `warmup` untimed steps.  The
    products rotate over the copies: step s runs A x on copy 2s and A^T x on
    copy 2s + 1 (mod the number of copies), so no product re-reads the
    arrays the one before it streamed.  HIP events at the two ends of each
    run, on the stream the kernels are launched on, with a synchronize on
    both sides."""
    ydt = plan.ytorch
    if not cp.y or cp.y[0].dtype != ydt:
        cp.outputs(torch, ydt)
    nc = len(cp.mats)

    def step(s):
        c = (2 * s) % nc
        C.csrc_spmv(cp.mats[c], plan, cp.x[c], cp.y[c])
        c = (2 * s + 1) % nc
        C.csrc_spmv_t(cp.mats[c], plan, cp.x[c], cp.yt[c])

    for s in range(warmup):
        step(s)
    out = []
    s0 = warmup
    stream = torch.cuda.current_stream()
    for _ in range(runs):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        for s in range(steps):
            step(s0 + s)
        t1.record(stream)
        torch.cuda.synchronize()
        s0 += steps
        out.append(t0.elapsed_time(t1) / steps)
    return out


def time_products(C, torch, cp, plan, count, transpose):
    """Mean ms per product over `count` back-to-back products of one kind
    (y = A x, or y = A^T x), HIP events only at the two ends."""
    nc = len(cp.mats)
    f = C.csrc_spmv_t if transpose else C.csrc_spmv
    out = cp.yt if transpose else cp.y
    for s in range(3):
        f(cp.mats[s % nc], plan, cp.x[s % nc], out[s % nc])
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for s in range(count):
        f(cp.mats[s % nc], plan, cp.x[s % nc], out[s % nc])
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1) / count


def kernel_source_hash(kind="single"):
    """Hash of the kernel sources of single-vector products, or of products
    with several right-hand sides (kind "multi"): paper_1003_0952_amd/sources.py."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("_csrc_sources", os.path.join(ROOT, "paper_1003_0952_amd",
                                                                                 "sources.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod.kernel_source_hash(kind)


def measured_traffic(workload, dtype, vname, vkw):
    """HBM bytes per product from the committed rocprofv3 counter summary, if it
    was taken on this kernel source and configuration; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{dtype}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("source_hash") != kernel_source_hash("multi" if workload.startswith("batch") else "single"):
        return None
    for e in d.get("entries", []):
        if e["variant"] == vname and e["options"] == vkw:
            return e["bytes_per_product"]
    return None


def hbm_ceiling(torch, C, nbytes=2 * 2**30, reps=5):
    """Measured ceilings (outside every timed region), each the median of 3
    runs of `reps` passes over nbytes: a read stream (the library's
    non-temporal 16-byte read kernel; every product here is an HBM read
    stream with a small write side) and a copy (bytes read + written)."""
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    sink = torch.zeros(65536, dtype=torch.int32, device="cuda")

    def rate(f, moved):
        f()
        torch.cuda.synchronize()
        runs = []
        for _ in range(3):
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(reps):
                f()
            t1.record()
            torch.cuda.synchronize()
            runs.append(moved * reps / (t0.elapsed_time(t1) * 1e-3) / 1e9)
        return round(float(np.median(runs)), 1)

    read = rate(lambda: C.csrc_stream_read(src, sink), nbytes)
    copy = rate(lambda: C.csrc_stream_copy(src, dst), 2 * nbytes)
    del src, dst, sink
    torch.cuda.empty_cache()
    return {"read_gbs": read, "copy_gbs": copy,
            "kind": f"hand-written read and copy kernels over {nbytes >> 20} MiB, median of 3 runs "
                    f"(copy counts bytes read + written)"}


def cpu_info():
    """CPU model, logical CPUs of the host and the CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count(), "allowed_cpus": len(os.sched_getaffinity(0))}


def pinned(f):
    """Run f() with this process pinned to one CPU (the first it may use),
    then restore the affinity.  Returns (f(), cpu)."""
    old = os.sched_getaffinity(0)
    cpu = min(old)
    os.sched_setaffinity(0, {cpu})
    try:
        return f(), cpu
    finally:
        os.sched_setaffinity(0, old)


def cpu_baseline(host, x, budget_s=12.0):
    """The oracle (plain sequential C, one thread pinned to one CPU) on the
    same matrix: steps of y = A x and y = A^T x.  Three runs of about
    budget_s / 3 each; returns (steps per run, median seconds per step, cpu)."""
    from oracle import reference as R
    c = {"n": host["n"], "k": host["k"], "ia": host["ia"], "ja": host["ja"],
         "ad": host["ad"], "al": host["al"], "au": host["au"]}

    def run():
        R.spmv(c, x)  # load / warm
        t0 = time.perf_counter()
        R.spmv(c, x)
        R.spmv_t(c, x)
        one = time.perf_counter() - t0
        reps = max(1, int(budget_s / 3 / max(one, 1e-6)))
        per = []
        for _ in range(3):
            t0 = time.perf_counter()
            for _ in range(reps):
                R.spmv(c, x)
                R.spmv_t(c, x)
            per.append((time.perf_counter() - t0) / reps)
        return reps, float(np.median(per))

    (reps, dt), cpu = pinned(run)
    return reps, dt, cpu


def bench_rect(args):
    """Rectangular matrices A = A_S + A_R (Sec. 2.1, Fig. 2b): the 27-point
    mesh of side^3 nodes plus couplings of its top face to side^2 overlap
    nodes (n x m, m = n + side^2).  A step is y = A x (x of m values) then
    y = A^T x (y of m values) on the next rotated copy; the square part runs
    under the given plan (default PRIVATE, atomic merge, 8192/256)."""
    import torch
    import paper_1003_0952_amd as C
    from synth import workloads as W
    from oracle import reference as R
    side = int(args.workload[4:] or 100)
    (n, m, rowptr, col, val), x = W.rect_mesh(side)
    (srp, scol, sval), r = C.csrc_rect_split(n, m, rowptr, col, val)
    host = C.csrc_from_csr(n, srp, scol, sval)
    k, kr = host["k"], r["kr"]
    vb = {"f64": 8, "f32": 4, "bf16": 2}[args.dtype]
    xb = 8 if args.dtype == "f64" else 4
    # square part (x and y of n values) plus A_R (iar, jar, ar) and the m - n
    # overlap values of x (or of y for the transpose)
    B1 = algorithmic_bytes(n, k, vb, xb, xb) + 4 * (n + 1) + kr * (4 + vb) + (m - n) * xb
    ncopy = args.copies or max(2, math.ceil(3 * MALL_BYTES / B1))
    mats = [C.Matrix(host, args.dtype) for _ in range(ncopy)]
    rps = [C.RectPart(r, args.dtype) for _ in range(ncopy)]
    if args.variant == "auto":
        vname, vkw = "private", {"tile_work": args.tile_work or 8192, "block": args.block or 256, "atomic_merge": 1}
    else:
        vname = args.variant
        vkw = {k_: v_ for k_, v_ in (("tile_work", args.tile_work), ("block", args.block),
                                     ("atomic_merge", args.atomic_merge)) if v_}
    plans = [C.Plan(A_, vname, **vkw) for A_ in mats]
    xd = mats[0].xdtype
    xs = [torch.from_numpy(x).to("cuda", xd) for _ in range(ncopy)]
    xts = [torch.from_numpy(x[:n]).to("cuda", xd) for _ in range(ncopy)]
    ys = [torch.empty(n, dtype=plans[0].ytorch, device="cuda") for _ in range(ncopy)]
    yts = [torch.empty(m, dtype=plans[0].ytorch, device="cuda") for _ in range(ncopy)]

    def step(s_):
        c = (2 * s_) % ncopy
        C.csrc_spmv_rect(mats[c], rps[c], plans[c], xs[c], ys[c])
        c = (2 * s_ + 1) % ncopy
        C.csrc_spmv_rect_t(mats[c], rps[c], plans[c], xts[c], yts[c])

    for s_ in range(args.warmup):
        step(s_)
    runs_ms = []
    for run in range(RUNS):
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        for s_ in range(args.steps):
            step(args.warmup + run * args.steps + s_)
        t1.record()
        torch.cuda.synchronize()
        runs_ms.append(t0.elapsed_time(t1) / args.steps)
    ms = float(np.median(runs_ms))
    c0 = R.csr_to_csrc(n, srp, scol, sval)
    C.csrc_spmv_rect(mats[0], rps[0], plans[0], xs[0], ys[0])
    C.csrc_spmv_rect_t(mats[0], rps[0], plans[0], xts[0], yts[0])
    torch.cuda.synchronize()

    def rel(a_, b_):
        return float(np.max(np.abs(a_ - b_)) / np.max(np.abs(b_)))

    err = max(rel(ys[0].double().cpu().numpy(), R.spmv_rect(c0, r, x)),
              rel(yts[0].double().cpu().numpy(), R.spmv_rect_t(c0, r, x[:n])))
    gbs = 2 * B1 / (ms * 1e-3) / 1e9
    nnz = 2 * k + n + kr
    out = {
        "metric": METRIC, "value": round(gbs, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "timing": f"median of {RUNS} runs of {args.steps} steps each", "ms_per_step_runs": [round(v, 5) for v in runs_ms],
        "warmup": args.warmup, "ms_per_step": round(ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": f"rect{side}_27pt_{args.dtype}", "n": n, "m": m, "nnz": nnz, "k": k, "kr": kr,
                   "variant": vname, **vkw, "copies": ncopy,
                   "step": "y=(A_S+A_R)x on copy 2s, then y=(A_S+A_R)^T x on copy 2s+1 (mod copies)"},
        "gflops": round(2 * (2 * (nnz - n) + n) / (ms * 1e-3) / 1e9, 1),
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "max_rel_err_vs_oracle": err,
        "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"rect{side}", args.dtype, vname, vkw),
                     "kernel": "one product = the square product's launches + k_rect_gather (or fill + k_rect_scatter)",
                     "bytes_per_launch": B1, "duration_us": round(ms / 2 * 1e3, 2)},
        "cpu_baseline": None,
    }
    print(json.dumps(out))


BATCH_COUNT = 256


def bench_batch(args):
    """Batched products: 256 seeded matrices (n log-uniform 1e3..2e5, 2-D
    9-point and 3-D 27-point patterns), each with 1..32 right-hand sides, in
    one persistent launch replayed as a HIP graph.  A step is Y = A X then
    Y = A^T X for every matrix of the batch (two graph launches)."""
    import torch
    import paper_1003_0952_amd as C
    from synth import workloads as W
    from paper_1003_0952_amd import tuner as T
    from oracle import reference as R

    t_setup = time.perf_counter()
    vb = {"f64": 8, "f32": 4, "bf16": 2}[args.dtype]
    xb = 8 if args.dtype == "f64" else 4
    ydt = "f64" if args.dtype == "f64" else "f32"
    members, mats, Xs = [], [], []
    B1 = F1 = 0
    nsum = ksum = 0
    for m in range(BATCH_COUNT):
        a, X = W.batch_member(m)
        host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
        A = C.Matrix(host, args.dtype)
        mats.append(A)
        Xs.append(torch.from_numpy(X).to("cuda", A.xdtype))
        members.append((a, X))
        r = X.shape[1]
        B1 += algorithmic_bytes(host["n"], host["k"], vb, xb, xb, r)
        F1 += flops(host["n"], host["k"], r)
        nsum += host["n"]
        ksum += host["k"]
    rs = [X.shape[1] for X in Xs]
    print(f"# setup {time.perf_counter() - t_setup:.1f}s matrices={BATCH_COUNT} rows={nsum} k={ksum} "
          f"bytes/product={B1}", file=sys.stderr, flush=True)

    def make(kw):
        bp = C.BatchPlan(mats, rs, ydtype=ydt, **kw)
        Ys = [torch.empty((A.n, r), dtype=bp.ytorch, device="cuda") for A, r in zip(mats, rs)]
        bp.bind(Xs, Ys)
        return bp, Ys, bp.graph(False), bp.graph(True)

    def time_graphs(g, gt, steps, warmup, runs=RUNS):
        """ms per step of `runs` timed runs of `steps` steps (forward graph
        then transpose graph), events at the two ends of each run."""
        for _ in range(warmup):
            C.BatchPlan.launch_graph(g)
            C.BatchPlan.launch_graph(gt)
        out = []
        for _ in range(runs):
            torch.cuda.synchronize()
            t0 = torch.cuda.Event(enable_timing=True)
            t1 = torch.cuda.Event(enable_timing=True)
            t0.record()
            for _ in range(steps):
                C.BatchPlan.launch_graph(g)
                C.BatchPlan.launch_graph(gt)
            t1.record()
            torch.cuda.synchronize()
            out.append(t0.elapsed_time(t1) / steps)
        return out

    # --- partition / tile shape: every batch candidate timed, fastest kept
    tuning = []
    best = None
    cands = T.BATCH_CANDIDATES
    if args.tile_work or args.block:
        cands = [{"variant": "private" if args.variant == "private" else "owner",
                  "tile_work": args.tile_work, "block": args.block}]
    for kw in cands:
        try:
            bp, Ys, g, gt = make(kw)
        except C.CsrcError as e:
            tuning.append({"candidate": kw, "error": str(e)})
            continue
        ms = float(np.median(time_graphs(g, gt, args.tune_steps, 2)))
        tuning.append({"candidate": kw, "ms_per_step": round(ms, 4)})
        print(f"# tune {kw} {ms:.4f} ms/step", file=sys.stderr, flush=True)
        if best is None or ms < best[1]:
            best = (kw, ms)
        del bp, Ys, g, gt
    kw = best[0]
    bp, Ys, g, gt = make(kw)
    runs_ms = time_graphs(g, gt, args.steps, args.warmup)
    ms = float(np.median(runs_ms))

    # parity spot check: the forward and transpose graphs on sampled members
    sample = sorted({0, 1, 64, 127, 128, 200, 254, 255, max(range(BATCH_COUNT), key=lambda i: mats[i].n)})
    err = {"Ax": 0.0, "ATx": 0.0}
    for tr, gg in ((False, g), (True, gt)):
        C.BatchPlan.launch_graph(gg)
        torch.cuda.synchronize()
        for i in sample:
            a, X = members[i]
            c = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
            f = R.spmv_t if tr else R.spmv
            ref = np.stack([f(c, np.ascontiguousarray(X[:, j])) for j in range(X.shape[1])], axis=1)
            got = Ys[i].double().cpu().numpy()
            e = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
            err["ATx" if tr else "Ax"] = max(err["ATx" if tr else "Ax"], e)

    cpu = None
    if not args.no_cpu:
        # passes over the members until about 12 s of products, pinned to one
        # CPU (only the products are timed, not the oracle's own CSRC split)
        def run_cpu():
            dt = 0.0
            done_b = 0
            done_m = 0
            split = {}
            while dt <= 12.0:
                for i in range(BATCH_COUNT):
                    a, X = members[i]
                    if i not in split:
                        split[i] = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
                    c = split[i]
                    t0 = time.perf_counter()
                    for j in range(X.shape[1]):
                        xj = np.ascontiguousarray(X[:, j])
                        R.spmv(c, xj)
                        R.spmv_t(c, xj)
                    dt += time.perf_counter() - t0
                    done_b += 2 * algorithmic_bytes(c["n"], c["k"], vb, xb, xb, X.shape[1])
                    done_m += 1
                    if dt > 12.0:
                        break
            return dt, done_b, done_m
        (dt, done_b, done_m), core = pinned(run_cpu)
        cpu = {"value": round(done_b / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"{done_m} members in batch order ({done_m / BATCH_COUNT:.2f} passes over the batch), "
                         f"every right-hand side, y=Ax and y=A^T x, "
                         f"plain sequential C oracle (FP64 values) pinned to CPU {core}, {dt:.1f} s",
               "pinned_cpu": core, **cpu_info()}

    gbs = 2 * B1 / (ms * 1e-3) / 1e9
    ach = gbs
    ceiling = hbm_ceiling(torch, C)
    ceiling["value_frac_of_read_ceiling"] = round(gbs / ceiling["read_gbs"], 4)
    out = {
        "metric": METRIC,
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "timing": f"median of {RUNS} runs of {args.steps} steps each",
        "ms_per_step_runs": [round(v, 5) for v in runs_ms],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"batch{BATCH_COUNT}_{args.dtype}", "matrices": BATCH_COUNT, "rows": nsum,
                   "k": ksum, "rhs_total": int(sum(rs)), **kw,
                   "step": "graph of Y=AX for all matrices, then graph of Y=A^T X"},
        "gflops": round(2 * F1 / (ms * 1e-3) / 1e9, 1),
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "max_rel_err_vs_oracle": err,
        "parity_sample": sample,
        "hbm_ceiling": ceiling,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(f"batch{BATCH_COUNT}", args.dtype, kw.get("variant", "owner"),
                                                 {k_: v_ for k_, v_ in kw.items() if k_ != "variant"}),
                     "kernel": ("one product = k_batch_pull (one graph launch)" if kw.get("variant", "owner") == "owner"
                                else "one product = k_batch_tiles + k_batch_merge (one graph launch)"),
                     "bytes_per_launch": B1, "duration_us": round(ms / 2 * 1e3, 2)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="hex100")
    ap.add_argument("--dtype", default="f64")
    ap.add_argument("--variant", default="auto", help="auto, or a variant name")
    ap.add_argument("--tile-work", type=int, default=0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--atomic-merge", type=int, default=0)
    ap.add_argument("--calibration-copy", action="store_true",
                    help="copy 256 MiB on the device three times first (counter calibration)")
    ap.add_argument("--lanes", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-pair", action="store_true", help="skip timing csrc_spmv_pair")
    ap.add_argument("--copies", type=int, default=0)
    ap.add_argument("--tune-steps", type=int, default=30)
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the product is "
                          "measured at one GPU's shard shape (see the design notes for sharding)"}))
        sys.exit(2)

    if args.calibration_copy:
        import torch
        src = torch.ones(2**25, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.workload.startswith("batch"):
        bench_batch(args)
        return
    if args.workload.startswith("rect"):
        bench_rect(args)
        return

    import torch
    import paper_1003_0952_amd as C

    t_setup = time.perf_counter()
    a, x = build_workload(args.workload)
    host = C.csrc_from_csr(a.n, a.rowptr, a.col, a.val)
    n, k = host["n"], host["k"]
    vb = {"f64": 8, "f32": 4, "bf16": 2}[args.dtype]
    xb = 8 if args.dtype == "f64" else 4
    yb = xb
    sym = args.workload.endswith("_sym")
    B1 = algorithmic_bytes(n, k, vb, xb, yb, symmetric=sym)
    ncopy = args.copies or max(2, math.ceil(3 * MALL_BYTES / B1))
    cp = Copies(C, torch, host, args.dtype, ncopy, x, symmetric=sym)
    print(f"# setup {time.perf_counter() - t_setup:.1f}s n={n} k={k} bytes/product={B1} copies={ncopy}",
          file=sys.stderr, flush=True)

    # --- variant choice (outside the timed region): the autotuner's pick; the
    # learned selector's pick for this matrix is reported with its regret
    from paper_1003_0952_amd import tuner as T, selector as S
    selection = {}
    tuning = []
    if args.variant == "auto":
        tuned = None
        tms = {}
        for i, (v, kw) in enumerate(T.CANDIDATES):
            if v in ("plain",):
                continue
            try:
                plan = C.Plan(cp.mats[0], v, **kw)
            except C.CsrcError as e:
                tuning.append({"candidate": T.candidate_name(i), "error": str(e)})
                continue
            ms = float(np.median(time_plan(C, torch, cp, plan, args.tune_steps, 3)))
            tms[i] = ms
            tuning.append({"candidate": T.candidate_name(i), "ms_per_step": round(ms, 4)})
            print(f"# tune {T.candidate_name(i)} {ms:.4f} ms/step", file=sys.stderr, flush=True)
            if tuned is None or ms < tuned[1]:
                tuned = (i, ms)
            del plan
        pick = tuned[0]
        selection = {"by": "autotuner", "candidate": T.candidate_name(pick)}
        model = S.Selector.load()
        if model is not None:
            lp = model.predict(C.csrc_features(host["ia"], host["ja"], args.dtype))
            selection["learned_pick"] = T.candidate_name(lp)
            if lp in tms:
                selection["learned_regret"] = round(tms[lp] / tuned[1] - 1.0, 4)
            d = T.DEFAULT if T.DEFAULT in tms else T.FALLBACK
            if d in tms:
                selection["default"] = T.candidate_name(d)
                selection["learned_gain_vs_default"] = round(tms[d] / tms.get(lp, tms[d]), 4)
        vname, vkw = T.CANDIDATES[pick][0], dict(T.CANDIDATES[pick][1])
    else:
        vname = args.variant
        vkw = {}
        if args.tile_work:
            vkw["tile_work"] = args.tile_work
        if args.block:
            vkw["block"] = args.block
        if args.atomic_merge:
            vkw["atomic_merge"] = args.atomic_merge
    if args.lanes:
        vkw["lanes"] = args.lanes
    plan = C.Plan(cp.mats[0], vname, **vkw)
    info = plan.info()

    # --- timed regions: three runs of back-to-back steps, events at the two
    # ends of each; the median run is the headline.  A product (all launches
    # of one y = A x or y = A^T x) takes half a step.
    runs_ms = time_plan(C, torch, cp, plan, args.steps, args.warmup)
    ms = float(np.median(runs_ms))
    per_prod_ms = ms / 2
    # the two product kinds apart, in passes of their own
    fwd = time_products(C, torch, cp, plan, min(args.steps, 50), False)
    bwd = time_products(C, torch, cp, plan, min(args.steps, 50), True)
    # warm: one copy reused, so part of it is served from the Infinity Cache
    # (reported beside the cache-cold headline, never as it)
    warm = time_products(C, torch, Copies.first(cp), plan, min(args.steps, 50), False)
    gbs = 2 * B1 / (ms * 1e-3) / 1e9
    gfl = 2 * flops(n, k) / (ms * 1e-3) / 1e9

    plain = None
    if not args.no_plain:
        pplan = C.Plan(cp.mats[0], "plain")
        pms = float(np.median(time_plan(C, torch, cp, pplan, max(10, args.steps // 4), 3)))
        plain = {"ms_per_step": round(pms, 4), "value": round(2 * B1 / (pms * 1e-3) / 1e9, 1),
                 "gflops": round(2 * flops(n, k) / (pms * 1e-3) / 1e9, 1),
                 "pct_hbm_peak": round(100 * 2 * B1 / (pms * 1e-3) / 1e9 / HBM_PEAK_GBS, 2)}

    # both products in one call (one pass over the entries when the plan is
    # PRIVATE with the atomic merge): time per pair against the step
    pair = None
    if not args.no_pair:
        nc = len(cp.mats)
        for s_ in range(3):
            C.csrc_spmv_pair(cp.mats[s_ % nc], plan, cp.x[s_ % nc], cp.y[s_ % nc], cp.yt[s_ % nc])
        torch.cuda.synchronize()
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        cnt = min(args.steps, 100)
        t0.record()
        for s_ in range(cnt):
            C.csrc_spmv_pair(cp.mats[s_ % nc], plan, cp.x[s_ % nc], cp.y[s_ % nc], cp.yt[s_ % nc])
        t1.record()
        torch.cuda.synchronize()
        pms_pair = t0.elapsed_time(t1) / cnt
        Bp = algorithmic_bytes(n, k, vb, xb, yb, symmetric=sym) + n * yb   # one more output vector
        pair = {"fused": bool(vname == "private" and vkw.get("atomic_merge")), "us_per_pair": round(pms_pair * 1e3, 2),
                "speedup_vs_two_products": round(ms / pms_pair, 3),
                "gbs": round(Bp / (pms_pair * 1e-3) / 1e9, 1), "bytes_per_pair": Bp}

    # parity spot check of the timed configuration against the oracle (and of
    # the pair call, when timed)
    # (the oracle splits the CSR input itself: no oracle input comes from the library)
    from oracle import reference as R
    c0 = R.csr_to_csrc(a.n, a.rowptr, a.col, a.val)
    ry = R.spmv(c0, x)
    ryt = R.spmv_t(c0, x)

    def rel(a_, b_):
        return float(np.max(np.abs(a_ - b_)) / np.max(np.abs(b_)))

    C.csrc_spmv(cp.mats[0], plan, cp.x[0], cp.y[0])
    C.csrc_spmv_t(cp.mats[0], plan, cp.x[0], cp.yt[0])
    torch.cuda.synchronize()
    err = max(rel(cp.y[0].double().cpu().numpy(), ry), rel(cp.yt[0].double().cpu().numpy(), ryt))
    if pair is not None:
        C.csrc_spmv_pair(cp.mats[0], plan, cp.x[0], cp.y[0], cp.yt[0])
        torch.cuda.synchronize()
        pair["max_rel_err_vs_oracle"] = max(rel(cp.y[0].double().cpu().numpy(), ry),
                                            rel(cp.yt[0].double().cpu().numpy(), ryt))

    cpu = None
    if not args.no_cpu:
        reps, dt, core = cpu_baseline(c0, x)
        cpu = {"value": round(2 * B1 / dt / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": f"full {args.workload} matrix, median of 3 runs of {reps} steps (y=Ax and y=A^T x "
                         f"each), plain sequential C oracle pinned to CPU {core}, {dt*1e3:.1f} ms/step",
               "gflops": round(2 * flops(n, k) / dt / 1e9, 3), "pinned_cpu": core, **cpu_info()}

    ach = B1 / (per_prod_ms * 1e-3) / 1e9
    ceiling = hbm_ceiling(torch, C)
    ceiling["value_frac_of_read_ceiling"] = round(gbs / ceiling["read_gbs"], 4)
    if vname == "private":
        launches = ("one product = k_fill_zero + k_private (atomic merge)" if vkw.get("atomic_merge")
                    else "one product = k_private + k_merge")
    else:
        launches = f"one product = all launches of the {vname} variant"
    traffic = measured_traffic(args.workload, args.dtype, vname, vkw)
    out = {
        "metric": METRIC,
        "value": round(gbs, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "timing": f"median of {RUNS} runs of {args.steps} steps each",
        "ms_per_step_runs": [round(v, 5) for v in runs_ms],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_27pt_{args.dtype}" if args.workload.startswith("hex")
                   else args.workload, "n": n, "nnz": 2 * k + n, "k": k, "variant": vname, **vkw,
                   "lanes": info["lanes"], "ntiles": info["ntiles"], "copies": ncopy,
                   "step": "y=Ax on copy 2s, then y=A^T x on copy 2s+1 (mod copies)"},
        "gflops": round(gfl, 1),
        "pct_hbm_peak": round(100 * gbs / HBM_PEAK_GBS, 2),
        "us_per_product": {"Ax": round(fwd * 1e3, 2), "ATx": round(bwd * 1e3, 2)},
        "warm_cache": {"us_per_product": round(warm * 1e3, 2), "gbs": round(B1 / (warm * 1e-3) / 1e9, 1),
                       "kind": "y=Ax on one copy reused (part of it served from the 256 MB Infinity "
                               "Cache); not the HBM figure"},
        "max_rel_err_vs_oracle": float(err),
        "hbm_ceiling": ceiling,
        "pair": pair,
        "plain_fp64": plain,
        "speedup_vs_plain": round(plain["ms_per_step"] / ms, 3) if plain else None,
        "selection": selection,
        "tuning": tuning,
        "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": launches, "bytes_per_launch": B1,
                     "duration_us": round(per_prod_ms * 1e3, 2)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()

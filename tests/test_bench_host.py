"""Host-side pieces of the benchmark: the byte and flop model, the traffic
summary lookup and the one-GPU guard (no GPU needed)."""

import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_algorithmic_bytes_match_the_working_set_model():
    """FP64, one right-hand side: 10 nnz + 18 n + 4 bytes (every array once),
    with nnz = 2k + n; the hexahedral benchmark matrix gives 282,635,924."""
    b = load_bench()
    n, k = 1_000_000, 12_731_796
    nnz = 2 * k + n
    assert b.algorithmic_bytes(n, k, 8, 8, 8) == 10 * nnz + 18 * n + 4 == 282_635_924
    # FP32 values, x and y: 6 nnz + 10 n + 4
    assert b.algorithmic_bytes(n, k, 4, 4, 4) == 6 * nnz + 10 * n + 4
    # one stored value array for numerically symmetric values
    assert b.algorithmic_bytes(n, k, 8, 8, 8, symmetric=True) == 282_635_924 - 8 * k
    # r right-hand sides: the vectors scale, the matrix is read once
    assert b.algorithmic_bytes(n, k, 8, 8, 8, r=4) == 282_635_924 + 3 * n * 16


def test_flops_count_two_nnz_minus_n():
    b = load_bench()
    n, k = 4096, 16002
    assert b.flops(n, k) == 2 * (2 * k + n) - n


def test_traffic_lookup_needs_the_current_kernel_source():
    """A counter summary is used only if it was taken on the kernel source
    as it is now and on the same configuration."""
    b = load_bench()
    path = os.path.join(ROOT, "profiles", "traffic_hex100_f64.json")
    with open(path) as fh:
        d = json.load(fh)
    e = d["entries"][0]
    got = b.measured_traffic("hex100", "f64", e["variant"], e["options"])
    if d["source_hash"] == b.kernel_source_hash("single"):
        assert got == e["bytes_per_product"]
        # reads at least the algorithmic bytes
        assert got >= d["algorithmic_bytes_per_product"]
    else:
        assert got is None
    assert b.measured_traffic("hex100", "f64", e["variant"], {"tile_work": 1}) is None
    assert b.measured_traffic("no_such_workload", "f64", e["variant"], e["options"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_package_exports_what_the_benchmark_and_smoke_use():
    """Every ``C.<name>`` that bench.py and the smoke entry call is exported
    by the package (a missing export only shows on the GPU otherwise)."""
    import re
    import paper_1003_0952_amd as C
    for f in ("bench.py", "__graft_entry__.py"):
        src = open(os.path.join(ROOT, f)).read()
        for name in sorted(set(re.findall(r"\bC\.([A-Za-z_][A-Za-z0-9_]*)", src))):
            assert hasattr(C, name), f"{f} uses C.{name}, which the package does not export"

"""Hashes of the kernel sources that decide a product's time and traffic.

Stored with every selector timing record and every committed traffic
summary; a record taken on other sources is stale and is not used.  Two
kinds: single-vector products (the tile, colour, atomic and plain kernels)
and products with several right-hand sides, batched ones included (the
owner multi-column kernels, their launch code and the batch plans).
"""

import hashlib
import os

_CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
_COMMON = ("csrc_plan.cpp", "internal.h", "device_common.h", "csrc_spmv.hip")
KERNEL_SOURCES = {
    "single": _COMMON,
    "multi": _COMMON + ("csrc_pull.hip", "csrc_batch.cpp"),
}


def kernel_source_hash(kind="single"):
    h = hashlib.sha1()
    for f in KERNEL_SOURCES[kind]:
        with open(os.path.join(_CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]

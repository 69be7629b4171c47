"""ctypes binding of libcsrc (argument marshalling only).

Every computation runs in the library: host-side setup in its C++ code, the
products in its HIP kernels.  torch supplies device memory and streams.  If
the shared library is missing this module raises at import: there is no
fallback path.
"""

import ctypes
import os

import numpy as np

# torch must be loaded first: its HIP runtime (soname libamdhip64.so.7) then
# satisfies libcsrc's dependency, so the process holds one HIP runtime and the
# library sees torch's devices, memory and streams.  Loading libcsrc first
# would pull a second runtime copy in beside torch's.
import torch  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libcsrc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"libcsrc.so not found at {LIB_PATH}: build it with "
        "`python paper_1003_0952_amd/build.py` (hipcc, gfx950)")

_lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
I32 = ctypes.c_int32
I64 = ctypes.c_int64
F32 = ctypes.c_float

# status codes (csrc.h)
OK = 0
ERR_ARG = -1
ERR_NOT_STRUCT_SYM = -2
ERR_DUPLICATE = -3
ERR_INDEX_RANGE = -4
ERR_TOO_LARGE = -5
ERR_ALIAS = -6
ERR_WORKSPACE = -7
ERR_HIP = -8
ERR_UNSUPPORTED = -9
ERR_PLAN = -10
ERR_NOMEM = -11
ERR_NO_MODEL = -12

F64, F32_, BF16 = 0, 1, 2
DTYPES = {"f64": F64, "f32": F32_, "bf16": BF16}

PLAIN, ATOMIC, PRIVATE, COLOR, OWNER, TILE_COLOR = 0, 1, 2, 3, 4, 5
VARIANTS = {"plain": PLAIN, "atomic": ATOMIC, "private": PRIVATE, "color": COLOR, "owner": OWNER,
            "tile_color": TILE_COLOR}
VARIANT_NAMES = {v: k for k, v in VARIANTS.items()}

PAD_PATTERN = 1
COLOR_WRITE_SET = 0
COLOR_DISTANCE2 = 1
NFEATURES = 12
NOALLOC_MAX_BYTES = 32 * 1024 * 1024   # CSRC_NOALLOC_MAX_BYTES


class CsrcError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        msg = _lib.csrc_status_string(status).decode()
        if status == ERR_HIP:
            msg += f" [{_lib.csrc_last_hip_error_string().decode()}]"
        super().__init__(f"{where}: {msg} ({status})" if where else f"{msg} ({status})")


def check(status, where=""):
    if status != OK:
        raise CsrcError(status, where)
    return status


class CsrcMatrix(ctypes.Structure):
    _fields_ = [("n", I32), ("vdtype", I32), ("k", I64), ("ia", P), ("ja", P),
                ("ad", P), ("al", P), ("au", P)]


class CsrcRect(ctypes.Structure):
    _fields_ = [("m", I32), ("vdtype", I32), ("kr", I64), ("iar", P), ("jar", P), ("ar", P)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("variant", I32), ("tile_work", I32), ("lanes", I32), ("block", I32),
                ("color_criterion", I32), ("ydtype", I32), ("compensated", I32),
                ("max_rhs", I32), ("persistent", I32), ("grid", I32),
                ("atomic_merge", I32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("variant", I32), ("ntiles", I32), ("ncolors", I32), ("lanes", I32),
                ("block", I32), ("max_tile_rows", I32), ("max_window", I32),
                ("nintervals", I32), ("window_slots", I64), ("pulled_rows", I64),
                ("lds_bytes", I64), ("workspace_bytes", I64)]


class BatchOpts(ctypes.Structure):
    _fields_ = [("tile_work", I32), ("block", I32), ("grid", I32), ("ydtype", I32), ("variant", I32)]


def _sig(name, res, args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = args
    return f


_sig("csrc_status_string", ctypes.c_char_p, [ctypes.c_int])
_sig("csrc_version", I32, [])
_sig("csrc_last_hip_error", I32, [])
_sig("csrc_last_hip_error_string", ctypes.c_char_p, [])
_sig("csrc_count", ctypes.c_int, [I32, P, P, I32, P])
_sig("csrc_from_csr", ctypes.c_int, [I32, P, P, P, I32, P, P, P, P, P])
_sig("csrc_rect_count", ctypes.c_int, [I32, I32, P, P, P, P])
_sig("csrc_rect_split", ctypes.c_int, [I32, I32, P, P, P, P, P, P, P, P, P])
_sig("csrc_spmv_rect", ctypes.c_int, [P, P, P, P, P, P, I64, P])
_sig("csrc_spmv_rect_t", ctypes.c_int, [P, P, P, P, P, P, I64, P])
_sig("csrc_quantize", ctypes.c_int, [I64, P, I32, P])
_sig("csrc_plan_opts_default", ctypes.c_int, [I32, P])
_sig("csrc_plan_create", ctypes.c_int, [I32, P, P, I32, P, P])
_sig("csrc_plan_destroy", ctypes.c_int, [P])
_sig("csrc_plan_workspace_bytes", I64, [P])
_sig("csrc_plan_upload", ctypes.c_int, [P, P, I64, P])
_sig("csrc_plan_get_info", ctypes.c_int, [P, P])
_sig("csrc_plan_export", ctypes.c_int, [P, I32, P, I64, P])
_sig("csrc_spmv", ctypes.c_int, [P, P, P, P, P, I64, P])
_sig("csrc_spmv_t", ctypes.c_int, [P, P, P, P, P, I64, P])
_sig("csrc_spmv_noalloc", ctypes.c_int, [P, P, P, P, P])
_sig("csrc_spmv_pair", ctypes.c_int, [P, P, P, P, P, P, I64, P])
_sig("csrc_spmm", ctypes.c_int, [P, P, I32, P, I64, P, I64, P, I64, P])
_sig("csrc_spmm_t", ctypes.c_int, [P, P, I32, P, I64, P, I64, P, I64, P])
_sig("csrc_batch_plan_create", ctypes.c_int, [I32, P, P, P, P, I32, P, P])
_sig("csrc_batch_plan_destroy", ctypes.c_int, [P])
_sig("csrc_batch_workspace_bytes", I64, [P])
_sig("csrc_batch_bind", ctypes.c_int, [P, P, P, P, P, P, P, I64, P])
_sig("csrc_batch_run", ctypes.c_int, [P, I32, P, I64, P])
_sig("csrc_spmv_batched", ctypes.c_int, [P, P, P, P, P, P, P, I64, P])
_sig("csrc_spmv_t_batched", ctypes.c_int, [P, P, P, P, P, P, P, I64, P])
_sig("csrc_batch_graph_create", ctypes.c_int, [P, I32, P, I64, P])
_sig("csrc_graph_launch", ctypes.c_int, [P, P])
_sig("csrc_graph_destroy", ctypes.c_int, [P])
_sig("csrc_color", ctypes.c_int, [I32, P, P, I32, P, P])
_sig("csrc_features", ctypes.c_int, [I32, P, P, I32, I32, P])
_sig("csrc_mlp_param_count", I64, [I32, I32])
_sig("csrc_mlp_forward", ctypes.c_int, [I32, I32, I32, P, P, P, P, P, P])
_sig("csrc_mlp_backward", ctypes.c_int, [I32, I32, I32, P, P, P, P, P, P, P, P, P])
_sig("csrc_mlp_predict_host", ctypes.c_int, [I32, I32, P, P, P, P, P])
_sig("csrc_select", ctypes.c_int, [I32, P, P, I32, I32, I32, P, P, P, P])
_sig("csrc_mlp_adam", ctypes.c_int, [I64, P, P, P, P, I32, F32, F32, F32, F32, P])
_sig("csrc_stream_read", ctypes.c_int, [P, I64, P, I32, P])
_sig("csrc_stream_copy", ctypes.c_int, [P, P, I64, I32, P])

lib = _lib


def np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


def t_ptr(t):
    """Device (or host) address of a torch tensor, as c_void_p."""
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)

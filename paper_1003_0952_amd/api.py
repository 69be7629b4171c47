"""Python face of libcsrc: the C entry points under the same names, plus
small owners (Matrix, Plan) that keep device buffers alive.

Nothing here computes: each function converts arguments and calls the
library.  Device memory comes from torch (ROCm) and streams are torch's.
"""

import ctypes

import numpy as np

from . import binding as B
from .binding import check, np_ptr, t_ptr, stream_ptr, CsrcError  # noqa: F401

_DT_NP = {B.F64: np.float64, B.F32_: np.float32, B.BF16: np.uint16}


def _dt(d):
    if isinstance(d, str):
        return B.DTYPES[d]
    return int(d)


def _variant(v):
    if isinstance(v, str):
        return B.VARIANTS[v]
    return int(v)


# ----------------------------------------------------------------- host side

def csrc_count(n, rowptr, col, pad=False):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    k = ctypes.c_int64(0)
    check(B.lib.csrc_count(int(n), np_ptr(rowptr), np_ptr(col), B.PAD_PATTERN if pad else 0,
                           ctypes.byref(k)), "csrc_count")
    return k.value


def csrc_from_csr(n, rowptr, col, val, pad=False):
    """CSR -> CSRC on the host (library code).  Returns dict of numpy arrays."""
    n = int(n)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    k = csrc_count(n, rowptr, col, pad)
    ia = np.zeros(n + 1, np.int32)
    ja = np.zeros(k, np.int32)
    ad = np.zeros(n, np.float64)
    al = np.zeros(k, np.float64)
    au = np.zeros(k, np.float64)
    check(B.lib.csrc_from_csr(n, np_ptr(rowptr), np_ptr(col), np_ptr(val),
                              B.PAD_PATTERN if pad else 0, np_ptr(ia), np_ptr(ja), np_ptr(ad),
                              np_ptr(al), np_ptr(au)), "csrc_from_csr")
    return {"n": n, "k": k, "ia": ia, "ja": ja, "ad": ad, "al": al, "au": au}


def csrc_rect_split(n, m, rowptr, col, val):
    """An n x m CSR matrix (m >= n) as A_S + A_R (Sec. 2.1), on the host
    (library code): returns (CSR of A_S as (rowptr, col, val), dict of A_R
    with n, m, kr, iar, jar, ar)."""
    n, m = int(n), int(m)
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    ns, nr = ctypes.c_int64(0), ctypes.c_int64(0)
    check(B.lib.csrc_rect_count(n, m, np_ptr(rowptr), np_ptr(col), ctypes.byref(ns), ctypes.byref(nr)),
          "csrc_rect_count")
    srp = np.zeros(n + 1, np.int64)
    scol = np.zeros(ns.value, np.int32)
    sval = np.zeros(ns.value, np.float64)
    iar = np.zeros(n + 1, np.int32)
    jar = np.zeros(nr.value, np.int32)
    ar = np.zeros(nr.value, np.float64)
    check(B.lib.csrc_rect_split(n, m, np_ptr(rowptr), np_ptr(col), np_ptr(val), np_ptr(srp), np_ptr(scol),
                                np_ptr(sval), np_ptr(iar), np_ptr(jar), np_ptr(ar)), "csrc_rect_split")
    return (srp, scol, sval), {"n": n, "m": m, "kr": int(nr.value), "iar": iar, "jar": jar, "ar": ar}


def csrc_quantize(a, dtype):
    d = _dt(dtype)
    a = np.ascontiguousarray(a, dtype=np.float64)
    out = np.empty(a.shape, dtype=_DT_NP[d])
    check(B.lib.csrc_quantize(a.size, np_ptr(a), d, np_ptr(out)), "csrc_quantize")
    return out


def csrc_color(ia, ja, criterion=B.COLOR_WRITE_SET):
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ja = np.ascontiguousarray(ja, dtype=np.int32)
    n = ia.shape[0] - 1
    col = np.zeros(n, np.int32)
    nc = ctypes.c_int32(0)
    check(B.lib.csrc_color(n, np_ptr(ia), np_ptr(ja), int(criterion), np_ptr(col),
                           ctypes.byref(nc)), "csrc_color")
    return col, nc.value


def csrc_features(ia, ja, vdtype="f64", ncolors=-1):
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ja = np.ascontiguousarray(ja, dtype=np.int32)
    f = np.zeros(B.NFEATURES, np.float32)
    check(B.lib.csrc_features(ia.shape[0] - 1, np_ptr(ia), np_ptr(ja), _dt(vdtype), int(ncolors),
                              np_ptr(f)), "csrc_features")
    return f


# ------------------------------------------------------- argument checks
#
# The library receives raw device pointers and sizes; a tensor of the wrong
# type, length, layout or device would make a kernel read or write past its
# buffer.  Every wrapper below checks its tensors here, before any launch.

def _same_device(t, dev, name):
    import torch
    want = torch.device(dev)
    if t.device.type != want.type or (want.index is not None and t.device.index != want.index):
        raise ValueError(f"{name} is on {t.device}, the matrix on {want}")


def _vector(t, n, dtype, dev, name):
    """t: a contiguous 1-D tensor of at least n elements of dtype on dev."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 1-D tensor")
    if t.numel() < n:
        raise ValueError(f"{name} has {t.numel()} elements, needs {n}")
    _same_device(t, dev, name)


def _block(t, n, r, dtype, dev, name):
    """t: an n x r (or longer) row-major 2-D block of dtype on dev whose
    columns are contiguous (stride(1) == 1) and rows at least r apart."""
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")
    if t.dim() != 2 or t.shape[0] < n or t.shape[1] != r:
        raise ValueError(f"{name} must be a 2-D block of at least {n} rows and exactly {r} columns, "
                         f"got {tuple(t.shape)}")
    if r > 0 and (t.stride(1) != 1 or t.stride(0) < r):
        raise ValueError(f"{name} must be row-major with contiguous rows (stride(1) == 1, stride(0) >= r)")
    _same_device(t, dev, name)


def _xdtype(vdtype):
    import torch
    return torch.float64 if vdtype == B.F64 else torch.float32


def _check_plan(A, plan):
    if plan.n != A.n or plan.vdtype != A.vdtype:
        raise ValueError("plan was made for another matrix (order or storage type differs)")


# --------------------------------------------------------------- device side

class Matrix:
    """A CSRC matrix in device memory (torch tensors) with its descriptor.

    ``host`` is the dict of csrc_from_csr; values are stored as ``dtype``
    ("f64", "f32" or "bf16"; rounded by csrc_quantize).  The host structure
    (ia, ja) is kept for plan creation.  ``symmetric=True`` stores a
    numerically symmetric matrix (au equal to al, checked) once: the
    descriptor's au is al.
    """

    def __init__(self, host, dtype="f64", device="cuda", symmetric=False):
        import torch
        self.n = int(host["n"])
        self.k = int(host["k"])
        self.vdtype = _dt(dtype)
        self.host_ia = np.ascontiguousarray(host["ia"], dtype=np.int32)
        self.host_ja = np.ascontiguousarray(host["ja"], dtype=np.int32)
        self.device = device
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.ia = t(self.host_ia)
        self.ja = t(self.host_ja)
        self.ad = t(csrc_quantize(host["ad"], self.vdtype))
        self.al = t(csrc_quantize(host["al"], self.vdtype))
        self.symmetric = bool(symmetric)
        if self.symmetric:
            if not np.array_equal(host["al"], host["au"]):
                raise ValueError("symmetric=True needs au equal to al")
            self.au = self.al
        else:
            self.au = t(csrc_quantize(host["au"], self.vdtype))
        self.desc = B.CsrcMatrix(self.n, self.vdtype, self.k, t_ptr(self.ia).value or 0,
                                 t_ptr(self.ja).value or 0, t_ptr(self.ad).value or 0,
                                 t_ptr(self.al).value or 0, t_ptr(self.au).value or 0)

    @property
    def xdtype(self):
        import torch
        return torch.float64 if self.vdtype == B.F64 else torch.float32

    def nbytes(self):
        vb = {B.F64: 8, B.F32_: 4, B.BF16: 2}[self.vdtype]
        nv = 1 if self.symmetric else 2
        return 4 * (self.n + 1) + self.k * (4 + nv * vb) + self.n * vb


class RectPart:
    """The auxiliary CSR part A_R of a rectangular matrix in device memory,
    stored as ``dtype`` like its square part."""

    def __init__(self, r, dtype="f64", device="cuda"):
        import torch
        self.n, self.m, self.kr = int(r["n"]), int(r["m"]), int(r["kr"])
        self.vdtype = _dt(dtype)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
        self.iar = t(np.asarray(r["iar"], dtype=np.int32))
        self.jar = t(np.asarray(r["jar"], dtype=np.int32))
        self.ar = t(csrc_quantize(r["ar"], self.vdtype))
        self.desc = B.CsrcRect(self.m, self.vdtype, self.kr, t_ptr(self.iar).value or 0,
                               t_ptr(self.jar).value or 0, t_ptr(self.ar).value or 0)


class Plan:
    """A product plan for one matrix structure with its uploaded workspace."""

    def __init__(self, A, variant="private", tile_work=0, lanes=0, block=0,
                 color_criterion=B.COLOR_WRITE_SET, ydtype="f32", compensated=False,
                 max_rhs=1, atomic_merge=0, stream=None):
        import torch
        self.variant = _variant(variant)
        opts = B.PlanOpts()
        check(B.lib.csrc_plan_opts_default(self.variant, ctypes.byref(opts)), "opts")
        opts.tile_work = int(tile_work)
        opts.lanes = int(lanes)
        opts.block = int(block) if block else opts.block
        opts.color_criterion = int(color_criterion)
        opts.ydtype = _dt(ydtype)
        opts.compensated = 1 if compensated else 0
        opts.max_rhs = int(max_rhs)
        opts.atomic_merge = int(atomic_merge)
        h = ctypes.c_void_p(0)
        check(B.lib.csrc_plan_create(A.n, np_ptr(A.host_ia), np_ptr(A.host_ja), A.vdtype,
                                     ctypes.byref(opts), ctypes.byref(h)), "csrc_plan_create")
        self._h = h
        self.n, self.vdtype = A.n, A.vdtype
        self.ydtype = B.F64 if A.vdtype == B.F64 else _dt(ydtype)
        self.ws_bytes = int(B.lib.csrc_plan_workspace_bytes(h))
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=A.device)
        if self.ws_bytes:
            check(B.lib.csrc_plan_upload(h, t_ptr(self.workspace), self.ws_bytes,
                                         stream_ptr(stream)), "csrc_plan_upload")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and B is not None and getattr(B, "lib", None) is not None:
            B.lib.csrc_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def info(self):
        i = B.PlanInfo()
        check(B.lib.csrc_plan_get_info(self._h, ctypes.byref(i)), "info")
        return {f: getattr(i, f) for f, _ in B.PlanInfo._fields_}

    def export(self, what):
        need = ctypes.c_int64(0)
        check(B.lib.csrc_plan_export(self._h, int(what), None, 0, ctypes.byref(need)), "export")
        out = np.zeros(need.value, np.int32)
        check(B.lib.csrc_plan_export(self._h, int(what), np_ptr(out), need.value,
                                     ctypes.byref(need)), "export")
        return out

    @property
    def ytorch(self):
        import torch
        return torch.float64 if self.ydtype == B.F64 else torch.float32


def csrc_spmv(A, plan, x, y, stream=None):
    """y <- A x (overwrites y).  Asynchronous on the stream."""
    _check_plan(A, plan)
    _vector(x, A.n, _xdtype(A.vdtype), A.device, "x")
    _vector(y, A.n, plan.ytorch, A.device, "y")
    check(B.lib.csrc_spmv(ctypes.byref(A.desc), plan.handle, t_ptr(x), t_ptr(y),
                          t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)), "csrc_spmv")
    return y


def csrc_spmv_t(A, plan, x, y, stream=None):
    """y <- A^T x (overwrites y).  Asynchronous on the stream."""
    _check_plan(A, plan)
    _vector(x, A.n, _xdtype(A.vdtype), A.device, "x")
    _vector(y, A.n, plan.ytorch, A.device, "y")
    check(B.lib.csrc_spmv_t(ctypes.byref(A.desc), plan.handle, t_ptr(x), t_ptr(y),
                            t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)), "csrc_spmv_t")
    return y


def csrc_spmv_noalloc(A, plan, x, y, stream=None):
    """y <- A x like csrc_spmv, with the plan's tables and partials in the
    library's static device array instead of the plan's workspace (no
    allocation in the call).  Asynchronous on the stream; calls that
    overlap on one device race."""
    _check_plan(A, plan)
    _vector(x, A.n, _xdtype(A.vdtype), A.device, "x")
    _vector(y, A.n, plan.ytorch, A.device, "y")
    check(B.lib.csrc_spmv_noalloc(ctypes.byref(A.desc), plan.handle, t_ptr(x), t_ptr(y), stream_ptr(stream)),
          "csrc_spmv_noalloc")
    return y


def csrc_spmv_pair(A, plan, x, y, yt, stream=None):
    """y <- A x and yt <- A^T x (one pass over the entries with a PRIVATE
    atomic-merge plan).  Asynchronous on the stream."""
    _check_plan(A, plan)
    _vector(x, A.n, _xdtype(A.vdtype), A.device, "x")
    _vector(y, A.n, plan.ytorch, A.device, "y")
    _vector(yt, A.n, plan.ytorch, A.device, "yt")
    check(B.lib.csrc_spmv_pair(ctypes.byref(A.desc), plan.handle, t_ptr(x), t_ptr(y), t_ptr(yt),
                               t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)), "csrc_spmv_pair")
    return y, yt


def csrc_spmv_rect(A, R, plan, x, y, stream=None):
    """y (n) <- (A_S + A_R) x (m), Fig. 2b.  Asynchronous on the stream."""
    _check_plan(A, plan)
    if R.vdtype != A.vdtype or R.n != A.n:
        raise ValueError("rectangular part does not match the matrix")
    _vector(x, R.m, _xdtype(A.vdtype), A.device, "x")
    _vector(y, A.n, plan.ytorch, A.device, "y")
    check(B.lib.csrc_spmv_rect(ctypes.byref(A.desc), ctypes.byref(R.desc), plan.handle, t_ptr(x), t_ptr(y),
                               t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)), "csrc_spmv_rect")
    return y


def csrc_spmv_rect_t(A, R, plan, x, y, stream=None):
    """y (m) <- (A_S + A_R)^T x (n).  Asynchronous on the stream."""
    _check_plan(A, plan)
    if R.vdtype != A.vdtype or R.n != A.n:
        raise ValueError("rectangular part does not match the matrix")
    _vector(x, A.n, _xdtype(A.vdtype), A.device, "x")
    _vector(y, R.m, plan.ytorch, A.device, "y")
    check(B.lib.csrc_spmv_rect_t(ctypes.byref(A.desc), ctypes.byref(R.desc), plan.handle, t_ptr(x), t_ptr(y),
                                 t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)), "csrc_spmv_rect_t")
    return y


def csrc_spmm(A, plan, X, Y, stream=None):
    """Y <- A X for row-major n x r blocks (torch 2-D tensors, row stride = ld)."""
    _check_plan(A, plan)
    r = X.shape[1] if X.dim() == 2 else -1
    _block(X, A.n, r, _xdtype(A.vdtype), A.device, "X")
    _block(Y, A.n, r, plan.ytorch, A.device, "Y")
    check(B.lib.csrc_spmm(ctypes.byref(A.desc), plan.handle, r, t_ptr(X), X.stride(0), t_ptr(Y),
                          Y.stride(0), t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)),
          "csrc_spmm")
    return Y


def csrc_spmm_t(A, plan, X, Y, stream=None):
    """Y <- A^T X for row-major n x r blocks."""
    _check_plan(A, plan)
    r = X.shape[1] if X.dim() == 2 else -1
    _block(X, A.n, r, _xdtype(A.vdtype), A.device, "X")
    _block(Y, A.n, r, plan.ytorch, A.device, "Y")
    check(B.lib.csrc_spmm_t(ctypes.byref(A.desc), plan.handle, r, t_ptr(X), X.stride(0), t_ptr(Y),
                            Y.stride(0), t_ptr(plan.workspace), plan.ws_bytes, stream_ptr(stream)),
          "csrc_spmm_t")
    return Y


def spmv(A, plan, x, y=None, transpose=False, stream=None):
    """Allocating convenience form of csrc_spmv / csrc_spmv_t."""
    import torch
    if y is None:
        y = torch.empty(A.n, dtype=plan.ytorch, device=x.device)
    return (csrc_spmv_t if transpose else csrc_spmv)(A, plan, x, y, stream)


# ------------------------------------------------------------------ batches

class BatchPlan:
    """Plan of many independent products run in one persistent launch.

    ``mats`` are Matrix objects of one storage type, ``rs`` their numbers of
    right-hand sides (1..32).  The workspace lives as long as the plan.
    """

    def __init__(self, mats, rs, tile_work=0, block=0, grid=0, ydtype="f32", variant="owner"):
        import torch
        self.mats = list(mats)
        self.rs = [int(r) for r in rs]
        m = len(self.mats)
        vd = self.mats[0].vdtype if m else B.F64
        n = np.array([a.n for a in self.mats], dtype=np.int32)
        self._ia = [a.host_ia for a in self.mats]
        self._ja = [a.host_ja for a in self.mats]
        ia_p = (ctypes.c_void_p * max(m, 1))(*[np_ptr(x).value for x in self._ia])
        ja_p = (ctypes.c_void_p * max(m, 1))(*[np_ptr(x).value for x in self._ja])
        r = np.array(self.rs, dtype=np.int32)
        if variant not in ("owner", "private"):
            raise ValueError("batch variant is 'owner' or 'private'")
        opts = B.BatchOpts(int(tile_work), int(block), int(grid), _dt(ydtype), B.VARIANTS[variant])
        self.variant = variant
        h = ctypes.c_void_p(0)
        check(B.lib.csrc_batch_plan_create(m, np_ptr(n), ia_p, ja_p, np_ptr(r), vd, ctypes.byref(opts),
                                           ctypes.byref(h)), "csrc_batch_plan_create")
        self._h = h
        self.vdtype = vd
        self.ydtype = B.F64 if vd == B.F64 else _dt(ydtype)
        self.ws_bytes = int(B.lib.csrc_batch_workspace_bytes(h))
        dev = self.mats[0].device if m else "cuda"
        self.workspace = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=dev)
        self._graphs = []

    def __del__(self):
        for g in getattr(self, "_graphs", []):
            if B is not None and getattr(B, "lib", None) is not None:
                B.lib.csrc_graph_destroy(g)
        h = getattr(self, "_h", None)
        if h is not None and h.value and B is not None and getattr(B, "lib", None) is not None:
            B.lib.csrc_batch_plan_destroy(h)
            self._h = None

    @property
    def ytorch(self):
        import torch
        return torch.float64 if self.ydtype == B.F64 else torch.float32

    def _arrays(self, Xs, Ys):
        m = len(self.mats)
        if len(Xs) != m or len(Ys) != m:
            raise ValueError(f"a batch of {m} matrices needs {m} X and {m} Y blocks")
        xdt = _xdtype(self.vdtype)
        for i, (A, r, X, Y) in enumerate(zip(self.mats, self.rs, Xs, Ys)):
            _block(X, A.n, r, xdt, A.device, f"X[{i}]")
            _block(Y, A.n, r, self.ytorch, A.device, f"Y[{i}]")
        descs = (B.CsrcMatrix * max(m, 1))(*[a.desc for a in self.mats])
        xp = (ctypes.c_void_p * max(m, 1))(*[t_ptr(x).value for x in Xs])
        yp = (ctypes.c_void_p * max(m, 1))(*[t_ptr(y).value for y in Ys])
        ldx = np.array([x.stride(0) for x in Xs], dtype=np.int64)
        ldy = np.array([y.stride(0) for y in Ys], dtype=np.int64)
        return descs, xp, ldx, yp, ldy

    def bind(self, Xs, Ys, stream=None):
        """Upload tables and the per-matrix pointers (X[m], Y[m]: n x r 2-D tensors)."""
        self._bound = (list(Xs), list(Ys))
        descs, xp, ldx, yp, ldy = self._arrays(Xs, Ys)
        check(B.lib.csrc_batch_bind(self._h, descs, xp, np_ptr(ldx), yp, np_ptr(ldy), t_ptr(self.workspace),
                                    self.ws_bytes, stream_ptr(stream)), "csrc_batch_bind")

    def run(self, transpose=False, stream=None):
        check(B.lib.csrc_batch_run(self._h, 1 if transpose else 0, t_ptr(self.workspace), self.ws_bytes,
                                   stream_ptr(stream)), "csrc_batch_run")

    def graph(self, transpose=False):
        """An instantiated HIP graph of the bound launch; call launch_graph(g)."""
        g = ctypes.c_void_p(0)
        check(B.lib.csrc_batch_graph_create(self._h, 1 if transpose else 0, t_ptr(self.workspace),
                                            self.ws_bytes, ctypes.byref(g)), "csrc_batch_graph_create")
        self._graphs.append(g)
        return g

    @staticmethod
    def launch_graph(g, stream=None):
        check(B.lib.csrc_graph_launch(g, stream_ptr(stream)), "csrc_graph_launch")


def csrc_spmv_batched(bplan, Xs, Ys, stream=None):
    """Bind then run Y[m] <- A[m] X[m] for every matrix of the batch plan."""
    bplan._bound = (list(Xs), list(Ys))
    descs, xp, ldx, yp, ldy = bplan._arrays(Xs, Ys)
    check(B.lib.csrc_spmv_batched(bplan._h, descs, xp, np_ptr(ldx), yp, np_ptr(ldy), t_ptr(bplan.workspace),
                                  bplan.ws_bytes, stream_ptr(stream)), "csrc_spmv_batched")


def csrc_spmv_t_batched(bplan, Xs, Ys, stream=None):
    """Bind then run Y[m] <- A[m]^T X[m] for every matrix of the batch plan."""
    bplan._bound = (list(Xs), list(Ys))
    descs, xp, ldx, yp, ldy = bplan._arrays(Xs, Ys)
    check(B.lib.csrc_spmv_t_batched(bplan._h, descs, xp, np_ptr(ldx), yp, np_ptr(ldy), t_ptr(bplan.workspace),
                                    bplan.ws_bytes, stream_ptr(stream)), "csrc_spmv_t_batched")


# -------------------------------------------------------------- measurement

def csrc_stream_read(src, sink, grid=0, stream=None):
    """Read the whole of device tensor src (non-temporal 16-byte loads);
    sink: uint32 device tensor of at least grid words (default grid: 8
    workgroups per compute unit)."""
    import torch
    nbytes = src.numel() * src.element_size()
    if grid <= 0:
        grid = 8 * torch.cuda.get_device_properties(src.device).multi_processor_count
    if sink.dtype != torch.int32 or sink.numel() < grid or sink.device != src.device:
        raise ValueError("sink must be an int32 tensor of at least grid elements on src's device")
    check(B.lib.csrc_stream_read(t_ptr(src), nbytes, t_ptr(sink), int(grid), stream_ptr(stream)),
          "csrc_stream_read")


def csrc_stream_copy(src, dst, grid=0, stream=None):
    """Copy device tensor src into dst (same byte size), non-temporal."""
    import torch
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or dst.device != src.device:
        raise ValueError("dst must have src's size and device")
    if grid <= 0:
        grid = 8 * torch.cuda.get_device_properties(src.device).multi_processor_count
    check(B.lib.csrc_stream_copy(t_ptr(src), t_ptr(dst), nbytes, int(grid), stream_ptr(stream)),
          "csrc_stream_copy")

"""MI355X (gfx950) CSRC sparse matrix-vector products.

Structurally symmetric sparse matrices stored in compressed sparse
row-column (CSRC) form: y = A x and the implicit transpose y = A^T x, in
hand-written HIP kernels behind the C ABI of ``include/csrc.h``
(``_lib/libcsrc.so``), with a ctypes binding of the same names here.
"""

from .api import (  # noqa: F401
    Matrix, Plan, csrc_count, csrc_from_csr, csrc_quantize, csrc_color, csrc_features,
    csrc_spmv, csrc_spmv_t, csrc_spmv_noalloc, csrc_spmv_pair, csrc_spmm, csrc_spmm_t, spmv,
    RectPart, csrc_rect_split, csrc_spmv_rect, csrc_spmv_rect_t,
    BatchPlan, csrc_spmv_batched, csrc_spmv_t_batched,
    csrc_stream_read, csrc_stream_copy,
)
from .binding import CsrcError, VARIANTS, VARIANT_NAMES, DTYPES  # noqa: F401

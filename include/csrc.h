/*
 * csrc.h -- C ABI of the MI355X (gfx950) CSRC sparse matrix-vector library.
 *
 * The operation (Batista, Ainsworth Jr., Ribeiro, "Parallel structurally-
 * symmetric sparse matrix-vector products on multi-core processors"):
 * given an n x n sparse matrix A with a structurally symmetric pattern and a
 * dense source vector x, compute the destination vector y = A x (Sec. 1), and
 * the transpose product y = A^T x that the format defines implicitly (Sec. 5).
 *
 * Storage (Sec. 2): A = A_D + A_L + A_U.
 *   ad[n]      diagonal entries a_ii (0 where not stored)
 *   ia[n+1]    row pointers of the strictly lower part (0-based, ia[0] = 0)
 *   ja[k]      column indices of the strictly lower part, ascending per row
 *   al[k]      al[q] = a(i, ja[q]) for q in row i          (A_L by rows)
 *   au[k]      au[q] = a(ja[q], i), the mirrored upper entry (A_U by columns)
 * k is the number of stored strictly-lower pairs.  Indices are int32.
 *
 * Conventions for every entry point:
 *   - The return value is a csrc_status; CSRC_OK (0) or a negative code.
 *     No C++ exception crosses the ABI.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *     memory of the current HIP device (the library never allocates or frees
 *     device memory: the caller passes buffers and a workspace).
 *   - stream is a hipStream_t passed as void*; NULL means the null stream.
 *     GPU entry points are asynchronous on that stream.
 *   - n = 0 is a valid no-op.  NaN and Inf propagate under IEEE rules.
 *   - Entry points are reentrant; a plan is immutable once created and may be
 *     shared by concurrent calls that use distinct workspaces.
 */
#ifndef CSRC_H
#define CSRC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
typedef enum csrc_status {
    CSRC_OK = 0,
    CSRC_ERR_ARG = -1,             /* null pointer, negative size, bad option   */
    CSRC_ERR_NOT_STRUCT_SYM = -2,  /* pattern of the input is not symmetric      */
    CSRC_ERR_DUPLICATE = -3,       /* an (i, j) pair stored twice                 */
    CSRC_ERR_INDEX_RANGE = -4,     /* column index outside [0, n)                 */
    CSRC_ERR_TOO_LARGE = -5,       /* k or a table does not fit 32-bit indices    */
    CSRC_ERR_ALIAS = -6,           /* destination overlaps the source             */
    CSRC_ERR_WORKSPACE = -7,       /* workspace null or smaller than required     */
    CSRC_ERR_HIP = -8,             /* a HIP runtime call failed                   */
    CSRC_ERR_UNSUPPORTED = -9,     /* variant cannot run this matrix (e.g. the
                                      private windows exceed the LDS budget)      */
    CSRC_ERR_PLAN = -10,           /* plan does not match the matrix or call      */
    CSRC_ERR_NOMEM = -11,          /* host allocation failed                      */
    CSRC_ERR_NO_MODEL = -12        /* csrc_select without a trained network: the
                                      caller tunes instead                        */
} csrc_status;

/* Human-readable name of a status code (static string, never NULL). */
const char *csrc_status_string(int status);

/* Library version as major*10000 + minor*100 + patch. */
int32_t csrc_version(void);

/* The hipError_t of the last HIP call that failed in this thread inside the
 * library (0 if none), and its name; they explain a CSRC_ERR_HIP. */
int32_t csrc_last_hip_error(void);
const char *csrc_last_hip_error_string(void);

/* ------------------------------------------------------------ data types */
typedef enum csrc_dtype {
    CSRC_F64 = 0,
    CSRC_F32 = 1,
    CSRC_BF16 = 2
} csrc_dtype;

/* ------------------------------------------------- host-side conversion */

/* Flags of csrc_count / csrc_from_csr. */
#define CSRC_PAD_PATTERN 1  /* add explicit zeros to symmetrise the pattern
                               instead of failing with CSRC_ERR_NOT_STRUCT_SYM */

/*
 * csrc_count -- validate a CSR matrix and count its strictly-lower pairs.
 * (Sec. 2: k = (nnz - n)/2 for a full diagonal; here k counts the stored
 * strictly-lower entries of the (possibly padded) symmetric pattern.)
 *   n        order of A (>= 0)
 *   row_ptr  host, n+1 entries, row_ptr[0] = 0, non-decreasing
 *   col      host, row_ptr[n] column indices (any order within a row)
 *   flags    0 or CSRC_PAD_PATTERN
 *   k_out    host, receives k
 * Errors: ARG, INDEX_RANGE, DUPLICATE, NOT_STRUCT_SYM, TOO_LARGE (k >= 2^31).
 */
int csrc_count(int32_t n, const int64_t *row_ptr, const int32_t *col,
               int32_t flags, int64_t *k_out);

/*
 * csrc_from_csr -- split a CSR matrix into CSRC arrays (Sec. 2).
 * All pointers are host memory owned by the caller.  Outputs: ia[n+1],
 * ja[k], ad[n], al[k], au[k] with k from csrc_count (same flags).  Within a
 * row the lower columns are sorted ascending, so the output is canonical.
 * Same errors as csrc_count.
 */
int csrc_from_csr(int32_t n, const int64_t *row_ptr, const int32_t *col,
                  const double *val, int32_t flags,
                  int32_t *ia, int32_t *ja, double *ad, double *al, double *au);

/*
 * Rectangular matrices (Sec. 2.1): an n x m matrix A with m >= n is
 * A_S + A_R, where A_S (n x n, the entries of columns < n) has a symmetric
 * pattern and goes to CSRC (csrc_count / csrc_from_csr on the square CSR
 * that csrc_rect_split writes) and A_R (the entries of columns >= n) stays
 * in CSR with global column indices.
 *
 * csrc_rect_count -- validate the n x m CSR (row_ptr[n+1], col) and count
 *   the entries of A_S (nnz_s) and of A_R (nnz_r).  Errors: ARG, INDEX_RANGE
 *   (a column outside [0, m)), TOO_LARGE (nnz_r >= 2^31).
 * csrc_rect_split -- write A_S as CSR (s_row_ptr[n+1], s_col[nnz_s],
 *   s_val[nnz_s]) and A_R as iar[n+1], jar[nnz_r], ar[nnz_r]; each row keeps
 *   its input order.  Host memory owned by the caller; same errors.
 */
int csrc_rect_count(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col,
                    int64_t *nnz_s, int64_t *nnz_r);
int csrc_rect_split(int32_t n, int32_t m, const int64_t *row_ptr, const int32_t *col,
                    const double *val, int64_t *s_row_ptr, int32_t *s_col, double *s_val,
                    int32_t *iar, int32_t *jar, double *ar);

/*
 * csrc_quantize -- round FP64 values to a storage type, host to host.
 *   dtype CSRC_F32: IEEE round-to-nearest-even; CSRC_BF16: RNE of the FP32
 *   value to bfloat16 (dst holds uint16 bit patterns); CSRC_F64: copy.
 */
int csrc_quantize(int64_t count, const double *src, int32_t dtype, void *dst);

/* ----------------------------------------------------------- matrices */

/* A CSRC matrix resident on the device.  Value arrays hold vdtype.  ja, al
 * and au must be 16-byte aligned (8-byte for BF16 values), as hipMalloc'd
 * memory is: the kernels read them with vector loads (CSRC_ERR_ARG if not).
 * Numerically symmetric storage (Sec. 2.2: a_ji = a_ij, so au equals al and
 * is not stored): pass au == al.  Every product then equals its transpose;
 * the PRIVATE single-vector kernels read al once per entry instead of two
 * value arrays, and the other kernels read the one array twice. */
typedef struct csrc_matrix {
    int32_t n;
    int32_t vdtype;        /* csrc_dtype of ad, al, au                        */
    int64_t k;
    const int32_t *ia;     /* device, n+1 */
    const int32_t *ja;     /* device, k   */
    const void *ad;        /* device, n   */
    const void *al;        /* device, k   */
    const void *au;        /* device, k   */
} csrc_matrix;

/*
 * Vector types.  FP64 storage uses FP64 x and y.  FP32/BF16 storage uses an
 * FP32 x and writes y as CSRC_F32 or CSRC_F64 (csrc_plan_opts.ydtype).  Its
 * products, per-lane row sums, window partials and the merge are FP32; the
 * per-tile sums in LDS that receive the scattered upper products are FP64
 * (gfx950 adds FP64 values in LDS at a far higher rate than FP32 ones), and
 * are rounded to the output type when they leave the tile.
 */

/* ------------------------------------------------------------ variants */
typedef enum csrc_variant {
    /* One thread per row; y cleared, then every row sum and every mirrored
       upper product added with a global atomic.  The plain baseline.        */
    CSRC_V_PLAIN = 0,
    /* Atomic scatter (Sec. 3: atomic primitives): y cleared, tiles stream
       ja/al/au; scatters below the tile are global atomic adds, scatters
       inside it and the row sums meet in LDS and are added to y with one
       global atomic per row.                                                  */
    CSRC_V_ATOMIC = 1,
    /* Local buffers (Sec. 3.1) per workgroup: a tile of nnz-balanced rows
       accumulates its own rows and its out-of-tile targets (its effective
       range, stored as compact windows) in LDS; pass 2 adds the windows into
       y in ascending tile order.                                              */
    CSRC_V_PRIVATE = 2,
    /* Colourful method (Sec. 3.2): rows grouped into conflict-free colour
       classes, processed one class per launch with plain stores; rows are
       walked by segments of g lanes (csrc_plan_opts.lanes) with the row sum
       reduced by lane shuffles.                                              */
    CSRC_V_COLOR = 3,
    /* Owner-computes: the workgroup that owns a tile of y also visits the
       rows above it that scatter into the tile, so every y entry is formed
       by one workgroup in LDS and stored once; no partials, no atomics.      */
    CSRC_V_OWNER = 4,
    /* Colour classes with a bounded stride (the refinement of the colourful
       method proposed in Sec. 5): the classes are built from tiles of
       consecutive rows (at most 2048) instead of single rows.  Each tile
       works in LDS as PRIVATE does; two tiles conflict iff the rows they
       write (their own rows and their window intervals) meet, and a greedy
       first-fit colouring in ascending tile order splits the tiles into
       conflict-free classes.  y is cleared, then one launch per class adds
       every tile's sums to y with plain read-modify-writes: no global
       atomics and no partial buffer.  The tiles' sums reach y in a fixed
       class order; inside a tile the LDS additions, as in every tile
       variant, come in the order the waves run.  One right-hand side
       (max_rhs 1).                                                           */
    CSRC_V_TILE_COLOR = 5,
    CSRC_V_COUNT = 6
} csrc_variant;

/* Colouring criteria (Sec. 3.2). */
#define CSRC_COLOR_WRITE_SET 0   /* rows conflict iff their write sets meet   */
#define CSRC_COLOR_DISTANCE2 1   /* direct or common-neighbour conflicts      */

typedef struct csrc_plan_opts {
    int32_t variant;          /* csrc_variant                                 */
    int32_t tile_work;        /* target work per tile, counted as 2 per lower
                                 pair + 1 per row (nnz-guided, Sec. 3.1);
                                 0 = default                                  */
    int32_t lanes;            /* lanes per row segment: 1,2,4,...,64; 0 = auto */
    int32_t block;            /* threads per workgroup: 64..1024, multiple of
                                 64; 0 = default                              */
    int32_t color_criterion;  /* CSRC_COLOR_*                                 */
    int32_t ydtype;           /* output type for FP32/BF16 storage            */
    int32_t compensated;      /* 1: compensated (TwoSum) accumulation of
                                 partial sums in the merge; reduced precision  */
    int32_t max_rhs;          /* largest r later passed to csrc_spmm (>= 1)   */
    int32_t persistent;       /* reserved, must be 0 (CSRC_ERR_ARG otherwise) */
    int32_t grid;             /* reserved, must be 0 (CSRC_ERR_ARG otherwise) */
    int32_t atomic_merge;     /* PRIVATE, one right-hand side:
                                 1 = y is cleared and every tile adds its own
                                 rows and its window sums to y with global
                                 atomics (no partial buffer, no merge pass;
                                 the order of the additions, hence the
                                 rounding, varies from run to run); 0 = window
                                 sums go to the partial buffer and a second
                                 pass adds them in tile order (deterministic) */
} csrc_plan_opts;

/* Fills opts with the defaults of a variant. */
int csrc_plan_opts_default(int32_t variant, csrc_plan_opts *opts);

typedef struct csrc_plan csrc_plan;   /* opaque, host-side */

/*
 * csrc_plan_create -- host-side setup for one matrix and one variant:
 * nnz-guided tiles (Sec. 3.1), effective-range windows and merge lists,
 * greedy colour classes (Sec. 3.2).  ia/ja are HOST copies of the matrix
 * structure.  vdtype is the storage type the plan will be used with.
 * Errors: ARG, UNSUPPORTED (e.g. windows beyond the LDS budget), NOMEM.
 */
int csrc_plan_create(int32_t n, const int32_t *ia, const int32_t *ja,
                     int32_t vdtype, const csrc_plan_opts *opts,
                     csrc_plan **out);
int csrc_plan_destroy(csrc_plan *plan);

/* Device workspace a plan needs (bytes, 256-byte aligned); 0 for none. */
int64_t csrc_plan_workspace_bytes(const csrc_plan *plan);

/*
 * csrc_plan_upload -- copy the plan's tables into the caller's device
 * workspace (ordered on stream).  Must precede the first product that uses
 * this workspace; the tables are then read-only, so one upload serves any
 * number of products.  Errors: WORKSPACE, HIP.
 */
int csrc_plan_upload(const csrc_plan *plan, void *workspace, int64_t bytes,
                     void *stream);

typedef struct csrc_plan_info {
    int32_t variant;
    int32_t ntiles;         /* workgroup tiles (0 for PLAIN)                   */
    int32_t ncolors;        /* colour classes (COLOR, TILE_COLOR)              */
    int32_t lanes;
    int32_t block;
    int32_t max_tile_rows;
    int32_t max_window;     /* largest per-tile window / pulled-row count      */
    int32_t nintervals;     /* window intervals over all tiles                 */
    int64_t window_slots;   /* partial slots over all tiles (PRIVATE)          */
    int64_t pulled_rows;    /* rows visited by non-owners (OWNER)              */
    int64_t lds_bytes;      /* dynamic LDS per workgroup                        */
    int64_t workspace_bytes;
} csrc_plan_info;

int csrc_plan_get_info(const csrc_plan *plan, csrc_plan_info *info);

/*
 * csrc_plan_export -- copy host-side plan tables (for verification):
 *   what 0: tile boundaries, ntiles+1 int32
 *   what 1: row colours, n int32 (COLOR); tile colours, ntiles int32
 *           (TILE_COLOR)
 *   what 2: window intervals, 3*nintervals int32 triples
 *           (tile, first row, row count), ascending by tile then row
 * count is the capacity of dst in int32 elements; the needed count is
 * returned in *needed.
 */
int csrc_plan_export(const csrc_plan *plan, int32_t what, int32_t *dst,
                     int64_t count, int64_t *needed);

/* --------------------------------------------------------------- products */

/*
 * csrc_spmv -- y <- A x (Fig. 2a semantics: y is overwritten, its input
 * contents are ignored).
 *   A          matrix descriptor (host struct holding device pointers)
 *   plan       from csrc_plan_create for this matrix structure
 *   x, y       device vectors of n elements (types above); y must not
 *              overlap x (CSRC_ERR_ALIAS)
 *   workspace  device buffer of csrc_plan_workspace_bytes(plan) bytes that
 *              holds the uploaded plan tables; NULL allowed when that size
 *              is 0
 * Errors: ARG, PLAN, ALIAS, WORKSPACE, HIP (launch failure).
 */
int csrc_spmv(const csrc_matrix *A, const csrc_plan *plan, const void *x,
              void *y, void *workspace, int64_t ws_bytes, void *stream);

/*
 * csrc_spmv_noalloc -- csrc_spmv without a workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The plan's tables and partial
 * buffer are placed in a static device array of the library,
 * CSRC_NOALLOC_MAX_BYTES per device, held from the library's load until the
 * process ends; each call copies the plan's tables into it (asynchronously
 * on stream: the plan must outlive the product) and then runs the kernels of
 * csrc_spmv.  No device or host memory is allocated.  Every call on a device
 * shares that device's array, so calls that overlap on one device (other
 * streams, other threads) race; serialise them.  Results equal csrc_spmv's
 * with the same plan.
 * Errors: as csrc_spmv; WORKSPACE when csrc_plan_workspace_bytes(plan)
 * exceeds CSRC_NOALLOC_MAX_BYTES (the 27-point 100^3 matrix needs 16 MiB
 * with PRIVATE 8192-work tiles and a merge pass, under 1 MiB with the atomic
 * merge).
 */
#define CSRC_NOALLOC_MAX_BYTES (32 * 1024 * 1024)
int csrc_spmv_noalloc(const csrc_matrix *A, const csrc_plan *plan, const void *x,
                      void *y, void *stream);

/* csrc_spmv_t -- y <- A^T x: the same kernels with al and au exchanged (Sec. 5). */
int csrc_spmv_t(const csrc_matrix *A, const csrc_plan *plan, const void *x,
                void *y, void *workspace, int64_t ws_bytes, void *stream);

/*
 * csrc_spmv_pair -- y <- A x and yt <- A^T x together (Sec. 5: the transpose
 * is the same loop with al and au exchanged; methods of the BiCG family need
 * both).  With a PRIVATE plan using the atomic merge (not persistent) one
 * pass reads ja, al and au once for both products; with any other plan, or
 * when the two sum arrays exceed the LDS, the two products run one after
 * the other.  x, y and yt are device vectors of n values (types as for
 * csrc_spmv) and must not overlap (CSRC_ERR_ALIAS).  Asynchronous on the
 * stream; errors as for csrc_spmv.
 */
int csrc_spmv_pair(const csrc_matrix *A, const csrc_plan *plan, const void *x,
                   void *y, void *yt, void *workspace, int64_t ws_bytes, void *stream);

/* The auxiliary CSR part A_R of a rectangular matrix, on the device: m
 * columns in total, kr entries, values of the matrix's vdtype. */
typedef struct csrc_rect {
    int32_t m;
    int32_t vdtype;
    int64_t kr;
    const int32_t *iar;    /* device, n+1 */
    const int32_t *jar;    /* device, kr; columns in [n, m) */
    const void *ar;        /* device, kr  */
} csrc_rect;

/*
 * csrc_spmv_rect -- y <- A x for A = A_S + A_R (Fig. 2b): x has m entries,
 *   y has n.  The square product of A (any plan) on x[0, n), then each row
 *   gathers its A_R entries from x.
 * csrc_spmv_rect_t -- y <- A^T x: x has n entries, y has m; y[0, n) is the
 *   square transpose product and y[n, m) receives A_R's entries scattered
 *   with atomics (the paper stops at A x; this is the transpose of the same
 *   matrix).
 * R->vdtype must equal A->vdtype; x and y must not overlap (CSRC_ERR_ALIAS).
 * Other arguments and errors as for csrc_spmv.
 */
int csrc_spmv_rect(const csrc_matrix *A, const csrc_rect *R, const csrc_plan *plan,
                   const void *x, void *y, void *workspace, int64_t ws_bytes, void *stream);
int csrc_spmv_rect_t(const csrc_matrix *A, const csrc_rect *R, const csrc_plan *plan,
                     const void *x, void *y, void *workspace, int64_t ws_bytes, void *stream);

/*
 * csrc_spmm / csrc_spmm_t -- Y <- A X (or A^T X) for r right-hand sides.
 * X and Y are row-major n x r blocks with leading dimensions ldx, ldy >= r
 * (element (i, c) at X[i*ldx + c]); 1 <= r <= plan max_rhs and r <= 32.
 * Each stored entry is read once and applied to all r columns.
 */
int csrc_spmm(const csrc_matrix *A, const csrc_plan *plan, int32_t r,
              const void *X, int64_t ldx, void *Y, int64_t ldy,
              void *workspace, int64_t ws_bytes, void *stream);
int csrc_spmm_t(const csrc_matrix *A, const csrc_plan *plan, int32_t r,
                const void *X, int64_t ldx, void *Y, int64_t ldy,
                void *workspace, int64_t ws_bytes, void *stream);

/* --------------------------------------------------------------- batches */

typedef struct csrc_batch_plan csrc_batch_plan;   /* opaque, host-side */

typedef struct csrc_batch_opts {
    int32_t tile_work;   /* target work per work item; 0 = default          */
    int32_t block;       /* threads per workgroup; 0 = default               */
    int32_t grid;        /* persistent workgroups; 0 = one per CU x occupancy */
    int32_t ydtype;      /* as csrc_plan_opts.ydtype                          */
    int32_t variant;     /* 0 or CSRC_V_OWNER: owner tiles, one launch;
                            CSRC_V_PRIVATE: local-buffer tiles + merge launch */
} csrc_batch_opts;

/*
 * csrc_batch_plan_create -- plan for nmat independent products in one
 * persistent launch.  Per matrix m: n[m], host structure ia[m], ja[m] and
 * its number of right-hand sides r[m] (1..32).
 *   OWNER (default): every matrix is cut into owner tiles; a lane group of
 *     G >= r lanes (a power of two, 4..32) holds a row's r columns, gathers
 *     the tile's rows in registers and pulls the scatters into the tile from
 *     the rows that make them (LDS sums), then stores Y once.  The work list
 *     is in matrix order, cut into eight ranges of equal cost, one per XCD.
 *     One kernel launch, no partial buffer.
 *   PRIVATE: local buffers of Sec. 3.1 in LDS, C columns at a time; window
 *     sums go to a partial buffer that a second launch merges; work list by
 *     decreasing cost.
 * Errors: ARG (bad r, n or variant), UNSUPPORTED (a tile's LDS exceeds the
 * budget), NOMEM, TOO_LARGE.
 */
int csrc_batch_plan_create(int32_t nmat, const int32_t *n,
                           const int32_t *const *ia, const int32_t *const *ja,
                           const int32_t *r, int32_t vdtype,
                           const csrc_batch_opts *opts, csrc_batch_plan **out);
int csrc_batch_plan_destroy(csrc_batch_plan *plan);
int64_t csrc_batch_workspace_bytes(const csrc_batch_plan *plan);

/*
 * csrc_batch_bind -- upload the plan tables and the per-matrix device
 * pointers (matrices A[0..nmat), blocks X[m], Y[m] with leading dimensions
 * ldx[m], ldy[m]) into the workspace.  Host arrays of nmat entries.
 */
int csrc_batch_bind(const csrc_batch_plan *plan, const csrc_matrix *A,
                    const void *const *X, const int64_t *ldx,
                    void *const *Y, const int64_t *ldy,
                    void *workspace, int64_t ws_bytes, void *stream);

/*
 * csrc_batch_run -- one persistent launch computing Y[m] <- A[m] X[m]
 * (transpose != 0: A[m]^T X[m]) for every bound matrix.  Launches kernels
 * only (no copies or memsets), so it may be captured into a HIP graph.
 */
int csrc_batch_run(const csrc_batch_plan *plan, int32_t transpose,
                   void *workspace, int64_t ws_bytes, void *stream);

/* Bind then run: the batched forms named after the single products. */
int csrc_spmv_batched(const csrc_batch_plan *plan, const csrc_matrix *A,
                      const void *const *X, const int64_t *ldx,
                      void *const *Y, const int64_t *ldy,
                      void *workspace, int64_t ws_bytes, void *stream);
int csrc_spmv_t_batched(const csrc_batch_plan *plan, const csrc_matrix *A,
                        const void *const *X, const int64_t *ldx,
                        void *const *Y, const int64_t *ldy,
                        void *workspace, int64_t ws_bytes, void *stream);

typedef struct csrc_graph csrc_graph;   /* opaque: an instantiated HIP graph */

/*
 * csrc_batch_graph_create -- build (not capture) a HIP graph whose kernel
 * nodes are the launches of csrc_batch_run with these arguments, in order
 * (one node for OWNER plans, two for PRIVATE);
 * csrc_graph_launch replays it on a stream.  The workspace must stay bound.
 */
int csrc_batch_graph_create(const csrc_batch_plan *plan, int32_t transpose,
                            void *workspace, int64_t ws_bytes,
                            csrc_graph **out);
int csrc_graph_launch(csrc_graph *graph, void *stream);
int csrc_graph_destroy(csrc_graph *graph);

/* ------------------------------------------------------------ colouring */

/*
 * csrc_color -- greedy first-fit colouring of the rows (Sec. 3.2), rows in
 * ascending index, each taking the smallest colour not held by an earlier
 * conflicting row.  Host memory.  color[n] receives the classes, *ncolors
 * their count.  criterion: CSRC_COLOR_WRITE_SET or CSRC_COLOR_DISTANCE2.
 */
int csrc_color(int32_t n, const int32_t *ia, const int32_t *ja,
               int32_t criterion, int32_t *color, int32_t *ncolors);

/* ------------------------------------------------- selection (learned) */

#define CSRC_NFEATURES 12

/*
 * csrc_features -- the 12 structural features the selector reads, from the
 * host structure (host memory):
 *   0 log2(n+1)            1 log2(nnz+1)         2 mean nnz/row
 *   3 var of nnz/row       4 max nnz/row / mean  5 bandwidth max|i-j| / n
 *   6 mean |i-j| / n       7 share of pairs with i-j < 64
 *   8 log2(1 + max writers of one y entry)       9 colours (write sets)/32
 *  10 log2(working-set bytes / 256 MiB)          11 3x3-block flag
 * ncolors < 0 makes the library colour the rows itself.
 */
int csrc_features(int32_t n, const int32_t *ia, const int32_t *ja,
                  int32_t vdtype, int32_t ncolors, float *features);

/*
 * Selector network (12-H-H-K MLP with ReLU and softmax cross-entropy), all
 * buffers on the device, FP32, row-major weight matrices W[out][in]:
 *   params layout: W1[H*12] b1[H] W2[H*H] b2[H] W3[K*H] b3[K]
 * csrc_mlp_param_count returns the number of floats in that layout.
 */
int64_t csrc_mlp_param_count(int32_t hidden, int32_t classes);

/*
 * csrc_mlp_forward -- logits[B*K] and probabilities probs[B*K] for a batch
 * of B feature rows feats[B*12] (device).  act may be NULL; otherwise it
 * receives the hidden activations [B*2H] needed by csrc_mlp_backward.
 * 1 <= hidden <= 256, 1 <= classes <= 64.  FP32, one workgroup per row.
 */
int csrc_mlp_forward(int32_t hidden, int32_t classes, int32_t batch,
                     const float *params, const float *feats, float *act,
                     float *logits, float *probs, void *stream);

/*
 * csrc_mlp_backward -- gradient grads[param_count] (device, overwritten) of
 * the mean softmax cross-entropy over the batch for integer labels[B]
 * (device, in [0, K)), and the loss itself in loss[0] (device; may be NULL).
 * Needs act and probs written by csrc_mlp_forward on the same batch and a
 * device work buffer of B*(2H+K) floats.  Every sum over the batch runs in a
 * fixed order, so equal inputs give bit-identical gradients.
 */
int csrc_mlp_backward(int32_t hidden, int32_t classes, int32_t batch,
                      const float *params, const float *feats,
                      const float *act, const float *probs,
                      const int32_t *labels, float *grads, float *loss,
                      float *work, void *stream);

/*
 * csrc_mlp_adam -- one Adam step (Kingma and Ba) on params with moment
 * buffers m, v (device, param_count floats each); step is 1-based.
 */
int csrc_mlp_adam(int64_t count, float *params, const float *grads, float *m,
                  float *v, int32_t step, float lr, float beta1, float beta2,
                  float eps, void *stream);

/*
 * csrc_mlp_predict_host -- inference on the host: standardise the 12
 * features as (f - mean) / scale, run the network (host memory, FP32) and
 * return the arg-max class in *cls (ties to the lower index).  Used to pick
 * a variant for a new matrix without any device work.
 */
int csrc_mlp_predict_host(int32_t hidden, int32_t classes, const float *params,
                          const float *mean, const float *scale,
                          const float *features, int32_t *cls);

/*
 * csrc_select -- the learned selector's pick for a matrix: the 12 features
 * of csrc_features (the library colours the rows), then csrc_mlp_predict_host.
 * ia/ja are HOST arrays (the structure of csrc_from_csr's output); params,
 * mean and scale a trained network in host memory (the layout of
 * csrc_mlp_param_count, 12 floats each for mean and scale).  *candidate is
 * the class index, i.e. the position in the candidate list the network was
 * trained on.  params == NULL returns CSRC_ERR_NO_MODEL without touching
 * *candidate: exhaustive tuning is the fallback, and it is the caller's --
 * it needs the matrix on the device and timed products, which this
 * host-only call does not have (the Python package's selector.choose times
 * every candidate when no model is present).  Errors: ARG, NOMEM.
 */
int csrc_select(int32_t n, const int32_t *ia, const int32_t *ja, int32_t vdtype,
                int32_t hidden, int32_t classes, const float *params, const float *mean,
                const float *scale, int32_t *candidate);

/* ------------------------------------------------------------ measurement */

/*
 * HBM ceiling probes (not part of the method): the rates that bound every
 * product here, which is an HBM read stream with a small write side.  The
 * paper states its products are bound by memory traffic (Sec. 4.1); these
 * calls measure what this device's memory delivers to one kernel.
 *
 * csrc_stream_read -- read bytes (a multiple of 16) of device memory src
 *   (16-byte aligned) with non-temporal 16-byte loads by grid workgroups of
 *   256 threads; workgroup b writes a checksum word to sink[b] (device,
 *   grid words), so no load can be dropped.  Asynchronous on stream.
 * csrc_stream_copy -- copy bytes (a multiple of 16) from src to dst (both
 *   16-byte aligned, not overlapping: CSRC_ERR_ALIAS) the same way.
 * Errors: ARG (null, misaligned, bytes not a multiple of 16, grid outside
 * 1..65536), ALIAS, HIP.
 */
int csrc_stream_read(const void *src, int64_t bytes, uint32_t *sink, int32_t grid, void *stream);
int csrc_stream_copy(const void *src, void *dst, int64_t bytes, int32_t grid, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CSRC_H */

// Internal declarations shared by the host and device sources of libcsrc.
#pragma once

#include <atomic>
#include <cstdint>
#include <cstddef>
#include <vector>
#include <new>

#include "../../include/csrc.h"

namespace csrc {

constexpr int kMaxRhs = 32;
constexpr int kMergeBlock = 256;      // rows per merge workgroup (PRIVATE)
constexpr int kMaxIntervals = 64;     // window intervals per PRIVATE tile
constexpr int64_t kLdsBudget = 160 * 1024;   // bytes of LDS per CU on gfx950

inline int64_t align256(int64_t b) { return (b + 255) & ~int64_t(255); }

inline int value_bytes(int32_t dt) { return dt == CSRC_F64 ? 8 : (dt == CSRC_F32 ? 4 : 2); }
inline int acc_bytes(int32_t vdt) { return vdt == CSRC_F64 ? 8 : 4; }
constexpr int64_t align16(int64_t b) { return (b + 15) & ~int64_t(15); }

constexpr int kMaxTileRows = 2048;   // rows per tile (per-row state lives in LDS)
constexpr int kPullRows = 1024;       // rows per pull chunk (OWNER)
constexpr int kPullEntries = 16384;   // stored entries per pull chunk (OWNER)

// Dynamic LDS of the flat tile kernels (acc = accumulator bytes).  The LDS
// sums that take scattered adds are FP64 for every storage type
// (kSumBytes).  x values come first, then the sums, each region 16-byte
// aligned (lds_xs); row ids of a block's entries are uint16, padded by 4.
//   PRIVATE: x of own rows then window slots, sums of own rows then window
//            slots (each sized by the largest rows + slots of one tile, smax);
//            row ids; one dummy sum per lane; window interval starts and slots
//   OWNER:   x of own rows and of pulled rows; sums of own rows; row ids
//   ATOMIC:  x, sums of own rows; row ids
constexpr int kSumBytes = 8;
constexpr int64_t lds_xs(int64_t n, int acc) { return align16(n * acc) + align16(n * kSumBytes); }
constexpr int kDummySums = 64;   // PRIVATE: one FP64 sum per lane that takes masked-off adds
inline int64_t lds_private(int64_t smax, int64_t emax, int64_t ivmax, int acc)
{
    return lds_xs(smax, acc) + align16((emax + 4) * 2) + kDummySums * kSumBytes + 2 * ivmax * 4;
}
// PRIVATE producing A x and A^T x together: the sums of both products
inline int64_t lds_private_pair(int64_t smax, int64_t emax, int64_t ivmax, int acc)
{
    return lds_xs(smax, acc) + align16(smax * kSumBytes) + align16((emax + 4) * 2) + 2 * ivmax * 4;
}
inline int64_t lds_owner(int64_t tmax, int64_t pmax, int64_t emax, int acc)
{
    return align16((tmax + pmax) * acc) + align16(tmax * kSumBytes) + align16((emax + 4) * 2);
}
inline int64_t lds_atomic(int64_t tmax, int64_t emax, int acc)
{
    return lds_xs(tmax, acc) + align16((emax + 4) * 2);
}
// multi-column forms: C columns of each per-row and per-slot array.  PRIVATE
// keeps them column-major with leading dimension mm_ld(smax), which is 1 mod
// 32 so that the C values of one row fall into different LDS banks.
constexpr int mm_ld(int64_t smax) { return (int)(((smax + 31) & ~int64_t(31)) + 1); }
inline int64_t lds_private_mm(int64_t smax, int64_t emax, int64_t ivmax, int acc, int C)
{
    return lds_xs((int64_t)mm_ld(smax) * C, acc) + align16((emax + 4) * 2) + 2 * ivmax * 4;
}
inline int mm_columns(int32_t vdtype) { return vdtype == CSRC_F64 ? 4 : 8; }

// Owner-computes multi-column kernel: a row's W columns (W a power of two,
// 4..32, at least r) are held by W / 4 lanes, four columns each; a tile's
// sums take rows x (W + 1) FP64 values of LDS (the odd leading dimension
// spreads the rows of concurrent groups over the banks), at most kOwnerMmLds
// bytes, so that four workgroups share a compute unit's 160 KiB.
constexpr int64_t kOwnerMmLds = 36 * 1024;
constexpr int mm_group(int r)
{
    int g = 4;
    while (g < r) g <<= 1;
    return g;
}
constexpr int owner_mm_ld(int w) { return w + 1; }
constexpr int owner_mm_max_rows(int g)
{
    return (int)(kOwnerMmLds / ((int64_t)owner_mm_ld(g) * 8)) < kMaxTileRows
               ? (int)(kOwnerMmLds / ((int64_t)owner_mm_ld(g) * 8))
               : kMaxTileRows;
}
inline int64_t lds_owner_pull(int64_t tmax, int g) { return tmax * owner_mm_ld(g) * 8; }

// A pull segment of an owner tile: entries [q0, q1) of row `row` (a row at
// or after the tile's first row) whose columns lie in the tile, i.e. the
// scatters row `row` makes into the tile.  16 bytes, read with one load.
struct alignas(16) PullSeg {
    int32_t row, q0, q1, pad;
};

// A table placed in the device workspace.
struct Table {
    int64_t offset = 0;   // bytes from the workspace base
    int64_t bytes = 0;
};

// Device-side view of a single-matrix plan (all pointers into the workspace).
// A run [lo, hi) of rows of one merge block covered by one window interval;
// row i's partial is partials[base + i].
struct MergeSeg {
    int32_t lo, hi;
    int64_t base;
};

// Per-tile record of a PRIVATE plan, 128 bytes read with scalar loads: the
// tile's rows [r0, r1) and entries [k0, k1), its window (ni intervals from
// global interval e0, w slots, partials from goff) and the first
// kRecIntervals intervals' first row and first slot (unused: INT32_MAX).
constexpr int kRecIntervals = 8;
struct TileRec {
    int32_t r0, r1, k0, k1;
    int32_t e0, ni, w;
    int32_t tail;   // the tile's entries end at the matrix's last one, an odd number of entries after
                    // k0 rounded down to even (a bfloat16 pair read there would reach past the array)
    int64_t goff;
    int32_t pad1[6];
    int32_t ivrow[kRecIntervals];
    int32_t ivslot[kRecIntervals];
};
static_assert(sizeof(TileRec) == 128, "tile record size");

struct PlanDev {
    const int32_t *tiles;      // ntiles+1 row boundaries
    const int32_t *tile_k;     // ntiles+1: ia at each boundary (first entry)
    const int32_t *iv_ptr;     // ntiles+1: intervals of each tile
    const int32_t *iv_row;     // first row of each interval
    const int32_t *iv_len;     // rows in each interval
    const int32_t *iv_slot;    // slot of the interval's first row in its tile window
    const int64_t *iv_goff;    // global partial offset of the interval's first row
    const TileRec *trec;       // PRIVATE: per-tile records
    const int32_t *mb_ptr;     // merge blocks: segments of each block
    const MergeSeg *mb_seg;
    const int32_t *crow;       // rows sorted by colour
    const int32_t *cptr;       // colour class boundaries (host copy used for launches)
    void *partials;            // partial buffer (PRIVATE)
    const int32_t *seg_ptr;    // OWNER: pull segments of each tile
    const PullSeg *segs;
};

// One bound matrix of a batch (written into the workspace by
// csrc_batch_bind): its arrays, blocks and plan tables.
struct MatDev {
    PlanDev P;
    int64_t k;
    const int32_t *ia;
    const int32_t *ja;
    const void *ad;
    const void *al;
    const void *au;
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    int32_t n;
    int32_t r;
    int32_t g;        // OWNER batches: columns per row W of the multi-column kernel
    int32_t pad;
};

// Parameter layout of the selector network (12-H-H-K perceptron): offsets
// of W1[H,12] b1[H] W2[H,H] b2[H] W3[K,H] b3[K] in one float array.
// constexpr, so host and device code share it.
constexpr int kMlpFeatures = CSRC_NFEATURES;
struct MlpLayout {
    int64_t W1, b1, W2, b2, W3, b3, total;
};
constexpr MlpLayout mlp_layout(int H, int K)
{
    MlpLayout L{};
    L.W1 = 0;
    L.b1 = L.W1 + (int64_t)H * kMlpFeatures;
    L.W2 = L.b1 + H;
    L.b2 = L.W2 + (int64_t)H * H;
    L.W3 = L.b2 + H;
    L.b3 = L.W3 + (int64_t)K * H;
    L.total = L.b3 + K;
    return L;
}
constexpr bool mlp_shape_ok(int H, int K, int B) { return H >= 1 && H <= 256 && K >= 1 && K <= 64 && B >= 0; }

}  // namespace csrc

struct csrc_plan {
    int32_t n = 0;
    int64_t k = 0;
    int32_t vdtype = CSRC_F64;
    csrc_plan_opts o{};
    int32_t ntiles = 0;
    int32_t max_tile_rows = 0;
    int32_t max_window = 0;     // PRIVATE: slots; OWNER: pulled rows
    int32_t max_span = 0;       // PRIVATE: largest rows + window slots of a tile
    int32_t max_intervals = 0;
    int32_t max_tile_entries = 0;   // stored lower entries of the largest tile
    int32_t max_pull_rows = 0;      // OWNER: rows of the largest pull chunk
    int32_t max_pull_entries = 0;   // OWNER: entries of the largest pull chunk
    int64_t window_slots = 0;
    int64_t pulled_rows = 0;
    int64_t lds_bytes = 0;
    int32_t ncolors = 0;
    int32_t nmerge_blocks = 0;
    // host tables
    std::vector<int32_t> tiles, tile_k, iv_ptr, iv_row, iv_len, iv_slot, mb_ptr;
    std::vector<csrc::MergeSeg> mb_seg;
    std::vector<csrc::TileRec> trec;
    std::vector<int64_t> iv_goff;
    std::vector<int32_t> color, crow, cptr;
    std::vector<int32_t> seg_ptr;          // OWNER: pull segments per tile
    std::vector<csrc::PullSeg> segs;
    int32_t mm_group = 0;                  // OWNER: columns per row W of the multi-column kernel
    // layout of the workspace
    csrc::Table t_tiles, t_tile_k, t_iv_ptr, t_iv_row, t_iv_len, t_iv_slot, t_iv_goff,
        t_mb_ptr, t_mb_seg, t_trec, t_crow, t_seg_ptr, t_segs, t_partials;
    int64_t blob_bytes = 0;      // bytes of uploaded tables (prefix of workspace)
    int64_t ws_bytes = 0;
    std::vector<char> blob;      // host image of the uploaded tables
};

namespace csrc {
// Records a failing HIP status for csrc_last_hip_error; returns CSRC_ERR_HIP
// (or CSRC_OK when status is 0).
int hip_status(int hip_error);
// host helpers implemented in csrc_host.cpp
int color_rows(int32_t n, const int32_t *ia, const int32_t *ja, int32_t criterion,
               int32_t *color, int32_t *ncolors);
// device view of a plan's tables uploaded at base (csrc_plan.cpp)
PlanDev plan_dev_at(const csrc_plan *p, char *base, char *partials);
// owner multi-column kernels (csrc_pull.hip): the single-matrix kernel for w
// columns per row (4, 8, 16 or 32) and the batched kernel, by storage and
// output type; nullptr for anything else
const void *owner_pull_kernel(int32_t vdtype, int32_t ydtype, int w);
const void *batch_pull_kernel(int32_t vdtype, int32_t ydtype);
}

// A batch of independent products: one PRIVATE plan per matrix, their tables
// concatenated into one workspace image with the work lists.
struct csrc_batch_plan {
    int32_t nmat = 0;
    int32_t vdtype = CSRC_F64;
    int32_t ydtype = CSRC_F64;
    csrc_batch_opts o{};
    std::vector<csrc_plan *> plans;
    std::vector<int32_t> n, r;
    std::vector<int64_t> blob_off;   // table image of matrix m in the workspace
    std::vector<int64_t> part_off;   // partial slots of matrix m (bytes, from off_parts)
    int32_t variant = CSRC_V_OWNER;  // OWNER (one pull kernel) or PRIVATE (tiles + merge)
    std::vector<int32_t> items;      // (matrix, tile) pairs: PRIVATE decreasing cost, OWNER matrix order
    std::vector<int32_t> mitems;     // (matrix, merge block) pairs (PRIVATE)
    std::vector<int32_t> xbeg;       // OWNER: 9 item boundaries, one range of equal cost per XCD
    int32_t smax = 0, emax = 0, ivmax = 0;   // largest rows + slots, entries, intervals of a tile
    int64_t lds = 0;
    std::vector<char> blob;          // tables + work lists (uploaded by bind)
    int64_t off_items = 0, off_mitems = 0, off_xbeg = 0, off_descs = 0, off_parts = 0, ws_bytes = 0;
    ~csrc_batch_plan()
    {
        for (auto *p : plans) delete p;
    }
};

struct csrc_graph {
    void *graph = nullptr;   // hipGraph_t
    void *exec = nullptr;    // hipGraphExec_t
};

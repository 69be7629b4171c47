// Host-side setup of a single-matrix product: nnz-guided tiles (Sec. 3.1),
// effective-range windows and merge lists for the local-buffer variant, pull
// lists for the owner-computes variant, colour classes (Sec. 3.2), and the
// layout of the tables in the caller's device workspace.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <vector>

#include "internal.h"

namespace {

int pow2_ceil(int v)
{
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// Lanes per row segment: smallest power of two covering the mean number of
// stored lower entries per row, within [2, 64].
int auto_lanes(int32_t n, int64_t k)
{
    if (n == 0) return 2;
    double mean = (double)k / n;
    int g = pow2_ceil((int)std::max(1.0, mean + 0.999));
    return std::min(64, std::max(2, g));
}

// Boundaries of `parts` contiguous row blocks of near-equal work, where row
// i weighs w_i = 2 (ia[i+1]-ia[i]) + 1: block b ends at the first row whose
// prefix work reaches (b+1)/parts of the total.
void nnz_partition(int32_t n, const int32_t *ia, int32_t parts, std::vector<int32_t> &s)
{
    s.assign(parts + 1, 0);
    int64_t total = 2 * (int64_t)ia[n] + n;
    int64_t prefix = 0;   // work of rows [0, i)
    int32_t b = 1;
    for (int32_t i = 0; i <= n && b < parts; ++i) {
        while (b < parts && prefix * parts >= (int64_t)b * total) s[b++] = i;
        if (i < n) prefix += 2 * (int64_t)(ia[i + 1] - ia[i]) + 1;
    }
    while (b < parts) s[b++] = n;
    s[parts] = n;
}

// Split blocks of more than max_rows rows into m = ceil(rows/max_rows)
// pieces at r0 + floor(p*rows/m): a tile keeps per-row state in LDS.
void cap_tile_rows(std::vector<int32_t> &s, int32_t max_rows)
{
    std::vector<int32_t> out;
    out.reserve(s.size());
    out.push_back(s[0]);
    for (size_t b = 0; b + 1 < s.size(); ++b) {
        int64_t r0 = s[b], rows = (int64_t)s[b + 1] - r0;
        int64_t m = std::max<int64_t>(1, (rows + max_rows - 1) / max_rows);
        for (int64_t q = 1; q <= m; ++q) out.push_back((int32_t)(r0 + (q * rows) / m));
    }
    s.swap(out);
}

// Sorted distinct rows -> intervals, merging gaps of at most `gap` rows.
void make_intervals(const std::vector<int32_t> &rows, int32_t gap,
                    std::vector<std::pair<int32_t, int32_t>> &iv)
{
    iv.clear();
    for (int32_t r : rows) {
        if (!iv.empty() && r - (iv.back().first + iv.back().second) <= gap)
            iv.back().second = r - iv.back().first + 1;
        else
            iv.push_back({r, 1});
    }
}

template <class T>
void put(std::vector<char> &blob, csrc::Table &t, const std::vector<T> &v)
{
    t.offset = (int64_t)blob.size();
    t.bytes = (int64_t)(v.size() * sizeof(T));
    blob.resize(csrc::align256(t.offset + std::max<int64_t>(t.bytes, 1)));
    if (t.bytes) std::memcpy(blob.data() + t.offset, v.data(), (size_t)t.bytes);
}

}  // namespace

extern "C" int csrc_plan_opts_default(int32_t variant, csrc_plan_opts *o)
{
    if (!o || variant < 0 || variant >= CSRC_V_COUNT) return CSRC_ERR_ARG;
    std::memset(o, 0, sizeof(*o));
    o->variant = variant;
    o->tile_work = 0;
    o->lanes = 0;
    o->block = 0;
    o->color_criterion = CSRC_COLOR_WRITE_SET;
    o->ydtype = CSRC_F32;
    o->compensated = 0;
    o->max_rhs = 1;
    return CSRC_OK;
}

static int default_tile_work(int32_t variant)
{
    switch (variant) {
    case CSRC_V_ATOMIC: return 8192;
    case CSRC_V_PRIVATE: return 8192;
    case CSRC_V_OWNER: return 16384;
    // a class holds about n / bandwidth tiles whatever their size: large
    // tiles keep the number of classes (launches) small
    case CSRC_V_TILE_COLOR: return 32768;
    default: return 4096;
    }
}

extern "C" int csrc_plan_create(int32_t n, const int32_t *ia, const int32_t *ja, int32_t vdtype,
                                const csrc_plan_opts *opts, csrc_plan **out)
{
    if (!out || !opts || n < 0 || (n > 0 && (!ia || (ia[n] > 0 && !ja)))) return CSRC_ERR_ARG;
    if (vdtype < CSRC_F64 || vdtype > CSRC_BF16) return CSRC_ERR_ARG;
    const csrc_plan_opts &o = *opts;
    if (o.variant < 0 || o.variant >= CSRC_V_COUNT) return CSRC_ERR_ARG;
    if (o.block != 0 && (o.block < 64 || o.block > (o.variant == CSRC_V_OWNER ? 1024 : 512) || o.block % 64))
        return CSRC_ERR_ARG;
    if (o.lanes != 0 && (o.lanes < 1 || o.lanes > 64 || (o.lanes & (o.lanes - 1)))) return CSRC_ERR_ARG;
    if (o.tile_work < 0 || o.max_rhs < 0 || o.max_rhs > csrc::kMaxRhs) return CSRC_ERR_ARG;
    if (o.persistent != 0 || o.grid != 0) return CSRC_ERR_ARG;   // reserved fields
    if (o.atomic_merge < 0 || o.atomic_merge > 1) return CSRC_ERR_ARG;
    if (o.atomic_merge && (o.variant != CSRC_V_PRIVATE || o.compensated)) return CSRC_ERR_ARG;
    if (o.variant == CSRC_V_TILE_COLOR && o.max_rhs > 1) return CSRC_ERR_ARG;
    if (vdtype != CSRC_F64 && o.ydtype != CSRC_F32 && o.ydtype != CSRC_F64) return CSRC_ERR_ARG;
    *out = nullptr;
    csrc_plan *p = nullptr;
    try {
        p = new csrc_plan();
        p->n = n;
        p->k = n ? ia[n] : 0;
        p->vdtype = vdtype;
        p->o = o;
        if (p->o.block == 0)
            // PRIVATE: 256 threads let six to eight tiles share a compute unit
            p->o.block = (o.variant == CSRC_V_PLAIN || o.variant == CSRC_V_COLOR ||
                          o.variant == CSRC_V_PRIVATE)
                             ? 256
                             : 512;
        if (p->o.lanes == 0) p->o.lanes = auto_lanes(n, p->k);
        if (p->o.lanes == 1) p->o.lanes = 2;
        if (p->o.tile_work == 0)
            p->o.tile_work = default_tile_work(o.variant) / (o.max_rhs > 1 ? 4 : 1);
        if (p->o.max_rhs == 0) p->o.max_rhs = 1;
        if (vdtype == CSRC_F64) p->o.ydtype = CSRC_F64;
        const int acc = csrc::acc_bytes(vdtype);
        const int v = p->o.variant;
        std::vector<char> &blob = p->blob;

        if (v != CSRC_V_PLAIN && v != CSRC_V_COLOR && n > 0) {
            int64_t total = 2 * p->k + n;
            int64_t parts = std::max<int64_t>(1, (total + p->o.tile_work - 1) / p->o.tile_work);
            if (parts > (int64_t)1 << 30) { delete p; return CSRC_ERR_TOO_LARGE; }
            nnz_partition(n, ia, (int32_t)parts, p->tiles);
            // the owner multi-column kernel keeps a tile's rows x r sums in LDS
            int32_t cap = csrc::kMaxTileRows;
            if (v == CSRC_V_OWNER) {
                p->mm_group = csrc::mm_group(p->o.max_rhs);
                cap = csrc::owner_mm_max_rows(p->mm_group);
            }
            cap_tile_rows(p->tiles, cap);
            // a tile is a non-empty block (more blocks than rows, or rows
            // heavier than a block's share, leave empty ones)
            p->tiles.erase(std::unique(p->tiles.begin(), p->tiles.end()), p->tiles.end());
            p->ntiles = (int32_t)p->tiles.size() - 1;
            p->tile_k.resize(p->tiles.size());
            for (size_t t = 0; t < p->tiles.size(); ++t) p->tile_k[t] = ia[p->tiles[t]];
            for (int32_t t = 0; t < p->ntiles; ++t) {
                p->max_tile_rows = std::max(p->max_tile_rows, p->tiles[t + 1] - p->tiles[t]);
                p->max_tile_entries = std::max(p->max_tile_entries, ia[p->tiles[t + 1]] - ia[p->tiles[t]]);
            }
            if (v == CSRC_V_ATOMIC) {
                p->lds_bytes = csrc::lds_atomic(p->max_tile_rows, p->max_tile_entries, acc);
                if (p->lds_bytes > csrc::kLdsBudget) { delete p; return CSRC_ERR_UNSUPPORTED; }
            }
        }

        const bool windows = v == CSRC_V_PRIVATE || v == CSRC_V_TILE_COLOR;
        if (windows && n > 0) {
            // Effective range of a tile (Sec. 3.1): its own rows plus the
            // rows below it that its loops write.  The latter are stored as a
            // few intervals (windows) whose slots hold the tile's partials.
            std::vector<int32_t> stamp(n, -1), tg;
            std::vector<std::pair<int32_t, int32_t>> iv;
            p->iv_ptr.assign(p->ntiles + 1, 0);
            int64_t slots = 0;
            for (int32_t t = 0; t < p->ntiles; ++t) {
                int32_t r0 = p->tiles[t], r1 = p->tiles[t + 1];
                tg.clear();
                for (int32_t q = ia[r0]; q < ia[r1]; ++q) {
                    int32_t j = ja[q];
                    if (j < r0 && stamp[j] != t) { stamp[j] = t; tg.push_back(j); }
                }
                std::sort(tg.begin(), tg.end());
                int32_t gap = 16;
                make_intervals(tg, gap, iv);
                while ((int)iv.size() > csrc::kMaxIntervals) {
                    gap *= 2;
                    make_intervals(tg, gap, iv);
                }
                int32_t w = 0;
                for (auto &e : iv) {
                    p->iv_row.push_back(e.first);
                    p->iv_len.push_back(e.second);
                    p->iv_slot.push_back(w);
                    p->iv_goff.push_back(slots + w);
                    w += e.second;
                }
                slots += w;
                p->iv_ptr[t + 1] = (int32_t)p->iv_row.size();
                p->max_window = std::max(p->max_window, w);
                p->max_span = std::max(p->max_span, p->tiles[t + 1] - p->tiles[t] + w);
                p->max_intervals = std::max(p->max_intervals, (int32_t)iv.size());
            }
            p->window_slots = slots;
            p->trec.resize(p->ntiles);
            for (int32_t t = 0; t < p->ntiles; ++t) {
                csrc::TileRec r{};
                r.r0 = p->tiles[t];
                r.r1 = p->tiles[t + 1];
                r.k0 = p->tile_k[t];
                r.k1 = p->tile_k[t + 1];
                r.e0 = p->iv_ptr[t];
                r.ni = p->iv_ptr[t + 1] - p->iv_ptr[t];
                r.w = r.ni ? p->iv_slot[r.e0 + r.ni - 1] + p->iv_len[r.e0 + r.ni - 1] : 0;
                r.goff = r.ni ? p->iv_goff[r.e0] : 0;
                r.tail = r.k1 == ia[n] && ((r.k1 - (r.k0 & ~1)) & 1);
                for (int k = 0; k < csrc::kRecIntervals; ++k) {
                    const bool in = k < r.ni;
                    r.ivrow[k] = in ? p->iv_row[r.e0 + k] : INT32_MAX;
                    r.ivslot[k] = in ? p->iv_slot[r.e0 + k] : INT32_MAX;
                }
                p->trec[t] = r;
            }
            // merge lists: for each block of kMergeBlock rows, the runs of
            // its rows covered by each interval, in ascending interval (=
            // tile) order
            int32_t nb = (n + csrc::kMergeBlock - 1) / csrc::kMergeBlock;
            p->nmerge_blocks = nb;
            p->mb_ptr.assign(nb + 1, 0);
            int32_t ni = (int32_t)p->iv_row.size();
            for (int32_t g = 0; g < ni; ++g) {
                int32_t b0 = p->iv_row[g] / csrc::kMergeBlock;
                int32_t b1 = (p->iv_row[g] + p->iv_len[g] - 1) / csrc::kMergeBlock;
                for (int32_t b = b0; b <= b1; ++b) p->mb_ptr[b + 1]++;
            }
            for (int32_t b = 0; b < nb; ++b) p->mb_ptr[b + 1] += p->mb_ptr[b];
            p->mb_seg.resize(p->mb_ptr[nb]);
            std::vector<int32_t> fill(p->mb_ptr.begin(), p->mb_ptr.end() - 1);
            for (int32_t g = 0; g < ni; ++g) {
                const int32_t a = p->iv_row[g], e = a + p->iv_len[g];
                int32_t b0 = a / csrc::kMergeBlock;
                int32_t b1 = (e - 1) / csrc::kMergeBlock;
                for (int32_t b = b0; b <= b1; ++b) {
                    csrc::MergeSeg sg;
                    sg.lo = std::max(a, b * csrc::kMergeBlock);
                    sg.hi = std::min(e, (b + 1) * csrc::kMergeBlock);
                    sg.base = p->iv_goff[g] - a;
                    p->mb_seg[fill[b]++] = sg;
                }
            }
            p->lds_bytes = csrc::lds_private(p->max_span, p->max_tile_entries, p->max_intervals, acc);
            if (p->o.max_rhs > 1)
                p->lds_bytes = std::max(p->lds_bytes,
                                        csrc::lds_private_mm(p->max_span, p->max_tile_entries, p->max_intervals,
                                                             acc, csrc::mm_columns(vdtype)));
            if (p->lds_bytes > csrc::kLdsBudget) { delete p; return CSRC_ERR_UNSUPPORTED; }
        }

        if (v == CSRC_V_TILE_COLOR && n > 0) {
            // Colour classes of tiles (the bounded-stride classes proposed in
            // Sec. 5).  The rows tile t writes are its own rows and every row
            // of its window intervals; rows -> writing tiles as a CSR filled
            // in ascending tile order, then greedy first-fit over the tiles.
            std::vector<int64_t> wptr((size_t)n + 1, 0);
            for (int32_t t = 0; t < p->ntiles; ++t) {
                for (int32_t r = p->tiles[t]; r < p->tiles[t + 1]; ++r) wptr[r + 1]++;
                for (int32_t g = p->iv_ptr[t]; g < p->iv_ptr[t + 1]; ++g)
                    for (int32_t r = p->iv_row[g]; r < p->iv_row[g] + p->iv_len[g]; ++r) wptr[r + 1]++;
            }
            for (int32_t i = 0; i < n; ++i) wptr[i + 1] += wptr[i];
            std::vector<int32_t> wt((size_t)wptr[n]);
            std::vector<int64_t> wfill(wptr.begin(), wptr.end() - 1);
            for (int32_t t = 0; t < p->ntiles; ++t) {
                for (int32_t r = p->tiles[t]; r < p->tiles[t + 1]; ++r) wt[wfill[r]++] = t;
                for (int32_t g = p->iv_ptr[t]; g < p->iv_ptr[t + 1]; ++g)
                    for (int32_t r = p->iv_row[g]; r < p->iv_row[g] + p->iv_len[g]; ++r) wt[wfill[r]++] = t;
            }
            p->color.assign(p->ntiles, 0);
            std::vector<int32_t> forbid;   // forbid[c] == t: colour c taken by a conflicting earlier tile
            p->ncolors = 0;
            auto visit = [&](int32_t t, int32_t r) {
                for (int64_t q = wptr[r]; q < wptr[r + 1] && wt[q] < t; ++q) forbid[p->color[wt[q]]] = t;
            };
            for (int32_t t = 0; t < p->ntiles; ++t) {
                if (forbid.size() < (size_t)p->ncolors + 1) forbid.resize((size_t)p->ncolors + 1, -1);
                for (int32_t r = p->tiles[t]; r < p->tiles[t + 1]; ++r) visit(t, r);
                for (int32_t g = p->iv_ptr[t]; g < p->iv_ptr[t + 1]; ++g)
                    for (int32_t r = p->iv_row[g]; r < p->iv_row[g] + p->iv_len[g]; ++r) visit(t, r);
                int32_t c = 0;
                while (forbid[c] == t) ++c;
                p->color[t] = c;
                p->ncolors = std::max(p->ncolors, c + 1);
            }
            p->cptr.assign(p->ncolors + 1, 0);
            for (int32_t t = 0; t < p->ntiles; ++t) p->cptr[p->color[t] + 1]++;
            for (int32_t c = 0; c < p->ncolors; ++c) p->cptr[c + 1] += p->cptr[c];
            p->crow.resize(p->ntiles);
            std::vector<int32_t> cf(p->cptr.begin(), p->cptr.end() - 1);
            for (int32_t t = 0; t < p->ntiles; ++t) p->crow[cf[p->color[t]]++] = t;
        }

        if (v == CSRC_V_OWNER && n > 0) {
            // Rows of later tiles that scatter into tile t, as intervals.
            std::vector<int32_t> tile_of(n);
            for (int32_t t = 0; t < p->ntiles; ++t)
                for (int32_t r = p->tiles[t]; r < p->tiles[t + 1]; ++r) tile_of[r] = t;
            std::vector<std::vector<int32_t>> pull(p->ntiles);
            for (int32_t i = 0; i < n; ++i) {
                int32_t ti = tile_of[i];
                int32_t last = -1;
                for (int32_t q = ia[i]; q < ia[i + 1]; ++q) {
                    int32_t tj = tile_of[ja[q]];
                    if (tj != ti && tj != last) {       // ja ascending -> tj ascending
                        pull[tj].push_back(i);
                        last = tj;
                    }
                }
            }
            std::vector<std::pair<int32_t, int32_t>> iv;
            p->iv_ptr.assign(p->ntiles + 1, 0);
            for (int32_t t = 0; t < p->ntiles; ++t) {
                make_intervals(pull[t], 4, iv);
                int32_t w = 0;
                for (auto &e : iv) {
                    // cut into chunks of at most kPullRows rows / kPullEntries
                    // entries (a single longer row stays one chunk)
                    int32_t a = e.first, end = e.first + e.second;
                    while (a < end) {
                        int32_t b = a + 1;
                        while (b < end && b - a < csrc::kPullRows &&
                               ia[b + 1] - ia[a] <= csrc::kPullEntries) ++b;
                        p->iv_row.push_back(a);
                        p->iv_len.push_back(b - a);
                        p->max_pull_rows = std::max(p->max_pull_rows, b - a);
                        p->max_pull_entries = std::max(p->max_pull_entries, ia[b] - ia[a]);
                        a = b;
                    }
                    w += e.second;
                }
                p->pulled_rows += w;
                p->iv_ptr[t + 1] = (int32_t)p->iv_row.size();
                p->max_window = std::max(p->max_window, w);
                p->max_intervals = std::max(p->max_intervals, (int32_t)iv.size());
                std::vector<int32_t>().swap(pull[t]);
            }
            const int64_t em = std::max(p->max_tile_entries, p->max_pull_entries);
            p->lds_bytes = csrc::lds_owner(p->max_tile_rows, p->max_pull_rows, em, acc);
            {
                // pull segments (products with strided or several right-hand
                // sides): for every row, each run of its entries (columns
                // ascending) that falls into one tile is a segment of that tile;
                // a tile's segments are in ascending row order
                p->seg_ptr.assign(p->ntiles + 1, 0);
                for (int32_t i = 0; i < n; ++i)
                    for (int32_t q = ia[i]; q < ia[i + 1]; ++q)
                        if (q == ia[i] || tile_of[ja[q]] != tile_of[ja[q - 1]]) p->seg_ptr[tile_of[ja[q]] + 1]++;
                for (int32_t t = 0; t < p->ntiles; ++t) p->seg_ptr[t + 1] += p->seg_ptr[t];
                p->segs.resize(p->seg_ptr[p->ntiles]);
                std::vector<int32_t> sf(p->seg_ptr.begin(), p->seg_ptr.end() - 1);
                for (int32_t i = 0; i < n; ++i) {
                    int32_t q = ia[i];
                    while (q < ia[i + 1]) {
                        const int32_t tj = tile_of[ja[q]];
                        int32_t e = q + 1;
                        while (e < ia[i + 1] && tile_of[ja[e]] == tj) ++e;
                        p->segs[sf[tj]++] = csrc::PullSeg{i, q, e, 0};
                        q = e;
                    }
                }
                p->lds_bytes = std::max(p->lds_bytes, csrc::lds_owner_pull(p->max_tile_rows, p->mm_group));
            }
            if (p->lds_bytes > csrc::kLdsBudget) { delete p; return CSRC_ERR_UNSUPPORTED; }
        }

        if (v == CSRC_V_COLOR && n > 0) {
            p->color.resize(n);
            int st = csrc::color_rows(n, ia, ja, p->o.color_criterion, p->color.data(), &p->ncolors);
            if (st) { delete p; return st; }
            p->cptr.assign(p->ncolors + 1, 0);
            for (int32_t i = 0; i < n; ++i) p->cptr[p->color[i] + 1]++;
            for (int32_t c = 0; c < p->ncolors; ++c) p->cptr[c + 1] += p->cptr[c];
            p->crow.resize(n);
            std::vector<int32_t> fill(p->cptr.begin(), p->cptr.end() - 1);
            for (int32_t i = 0; i < n; ++i) p->crow[fill[p->color[i]]++] = i;
        }

        // workspace image
        put(blob, p->t_tiles, p->tiles);
        put(blob, p->t_tile_k, p->tile_k);
        put(blob, p->t_iv_ptr, p->iv_ptr);
        put(blob, p->t_iv_row, p->iv_row);
        put(blob, p->t_iv_len, p->iv_len);
        put(blob, p->t_iv_slot, p->iv_slot);
        put(blob, p->t_iv_goff, p->iv_goff);
        put(blob, p->t_mb_ptr, p->mb_ptr);
        put(blob, p->t_mb_seg, p->mb_seg);
        put(blob, p->t_trec, p->trec);
        put(blob, p->t_crow, p->crow);
        put(blob, p->t_seg_ptr, p->seg_ptr);
        put(blob, p->t_segs, p->segs);
        p->blob_bytes = (int64_t)blob.size();
        p->t_partials.offset = p->blob_bytes;
        // the atomic merge of single products needs no partials
        p->t_partials.bytes = ((p->o.atomic_merge && p->o.max_rhs == 1) || v == CSRC_V_TILE_COLOR)
                                  ? 0
                                  : p->window_slots * acc * p->o.max_rhs;
        p->ws_bytes = csrc::align256(p->blob_bytes + p->t_partials.bytes);
        if (v == CSRC_V_PLAIN) p->ws_bytes = 0;
        *out = p;
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        delete p;
        return CSRC_ERR_NOMEM;
    }
}

extern "C" int csrc_plan_destroy(csrc_plan *p)
{
    delete p;
    return CSRC_OK;
}

extern "C" int64_t csrc_plan_workspace_bytes(const csrc_plan *p) { return p ? p->ws_bytes : -1; }

extern "C" int csrc_plan_upload(const csrc_plan *p, void *ws, int64_t bytes, void *stream)
{
    if (!p) return CSRC_ERR_ARG;
    if (p->ws_bytes == 0) return CSRC_OK;
    if (!ws || bytes < p->ws_bytes) return CSRC_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int st = csrc::hip_status(hipMemcpyAsync(ws, p->blob.data(), (size_t)p->blob_bytes,
                                             hipMemcpyHostToDevice, s));
    if (st) return st;
    // the host image stays owned by the plan; wait so callers may reuse it freely
    return csrc::hip_status(hipStreamSynchronize(s));
}

extern "C" int csrc_plan_get_info(const csrc_plan *p, csrc_plan_info *info)
{
    if (!p || !info) return CSRC_ERR_ARG;
    info->variant = p->o.variant;
    info->ntiles = p->ntiles;
    info->ncolors = p->ncolors;
    info->lanes = p->o.lanes;
    info->block = p->o.block;
    info->max_tile_rows = p->max_tile_rows;
    info->max_window = p->max_window;
    info->nintervals = (int32_t)p->iv_row.size();
    info->window_slots = p->window_slots;
    info->pulled_rows = p->pulled_rows;
    info->lds_bytes = p->lds_bytes;
    info->workspace_bytes = p->ws_bytes;
    return CSRC_OK;
}

extern "C" int csrc_plan_export(const csrc_plan *p, int32_t what, int32_t *dst, int64_t count,
                                int64_t *needed)
{
    if (!p || !needed) return CSRC_ERR_ARG;
    std::vector<int32_t> v;
    if (what == 0) {
        v = p->tiles;
    } else if (what == 1) {
        v = p->color;
    } else if (what == 2) {
        for (int32_t t = 0; t < (int32_t)p->iv_ptr.size() - 1; ++t)
            for (int32_t g = p->iv_ptr[t]; g < p->iv_ptr[t + 1]; ++g) {
                v.push_back(t);
                v.push_back(p->iv_row[g]);
                v.push_back(p->iv_len[g]);
            }
    } else {
        return CSRC_ERR_ARG;
    }
    *needed = (int64_t)v.size();
    if (count < (int64_t)v.size()) return dst ? CSRC_ERR_ARG : CSRC_OK;
    if (!v.empty()) std::memcpy(dst, v.data(), v.size() * 4);
    return CSRC_OK;
}

namespace csrc {

// Device pointers of a plan's tables placed at base (its uploaded image) and
// of its partial buffer.
PlanDev plan_dev_at(const csrc_plan *p, char *base, char *partials)
{
    auto at = [&](const Table &t) -> const void * { return base ? base + t.offset : nullptr; };
    PlanDev d;
    d.tiles = (const int32_t *)at(p->t_tiles);
    d.tile_k = (const int32_t *)at(p->t_tile_k);
    d.iv_ptr = (const int32_t *)at(p->t_iv_ptr);
    d.iv_row = (const int32_t *)at(p->t_iv_row);
    d.iv_len = (const int32_t *)at(p->t_iv_len);
    d.iv_slot = (const int32_t *)at(p->t_iv_slot);
    d.iv_goff = (const int64_t *)at(p->t_iv_goff);
    d.mb_ptr = (const int32_t *)at(p->t_mb_ptr);
    d.mb_seg = (const MergeSeg *)at(p->t_mb_seg);
    d.trec = (const TileRec *)at(p->t_trec);
    d.crow = (const int32_t *)at(p->t_crow);
    d.cptr = nullptr;
    d.partials = partials;
    d.seg_ptr = (const int32_t *)at(p->t_seg_ptr);
    d.segs = (const PullSeg *)at(p->t_segs);
    return d;
}

}  // namespace csrc

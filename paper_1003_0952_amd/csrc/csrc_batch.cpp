// Host-side setup of batched products: an OWNER (or PRIVATE) plan per
// matrix, their tables concatenated, and the work lists of the persistent
// launch.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace {

void put_ints(csrc_batch_plan *b, const std::vector<int32_t> &v, int64_t &off)
{
    off = (int64_t)b->blob.size();
    b->blob.resize(csrc::align256(off + std::max<int64_t>(1, (int64_t)v.size() * 4)));
    if (!v.empty()) std::memcpy(b->blob.data() + off, v.data(), v.size() * 4);
}

// OWNER batch: an owner plan per matrix (lane group G >= r, pull segments),
// the (matrix, tile) items in matrix order and the eight equal-cost ranges,
// one per XCD.  A tile's cost is its stored entries and rows times G.
int owner_batch(csrc_batch_plan *b, int32_t nmat, const int32_t *n, const int32_t *const *ia,
                const int32_t *const *ja, const int32_t *r, int32_t vdtype)
{
    std::vector<int64_t> cost;
    for (int32_t m = 0; m < nmat; ++m) {
        if (r[m] < 1 || r[m] > csrc::kMaxRhs || n[m] < 0) return CSRC_ERR_ARG;
        csrc_plan_opts po;
        csrc_plan_opts_default(CSRC_V_OWNER, &po);
        po.tile_work = b->o.tile_work;
        po.block = b->o.block;
        po.ydtype = b->ydtype;
        po.max_rhs = std::max(2, (int)r[m]);   // a lane group of at least four lanes
        csrc_plan *p = nullptr;
        int st = csrc_plan_create(n[m], ia[m], ja[m], vdtype, &po, &p);
        if (st) return st;
        b->plans.push_back(p);
        b->n.push_back(n[m]);
        b->r.push_back(r[m]);
        b->part_off.push_back(0);
        b->lds = std::max(b->lds, csrc::lds_owner_pull(p->max_tile_rows, p->mm_group));
        for (int32_t t = 0; t < p->ntiles; ++t) {
            const int64_t e = (int64_t)p->tile_k[t + 1] - p->tile_k[t];
            const int64_t rows = (int64_t)p->tiles[t + 1] - p->tiles[t];
            b->items.push_back(m);
            b->items.push_back(t);
            cost.push_back((2 * e + rows) * p->mm_group);
        }
    }
    if (b->lds > csrc::kLdsBudget) return CSRC_ERR_UNSUPPORTED;
    const int64_t nit = (int64_t)cost.size();
    if (nit >= ((int64_t)1 << 31)) return CSRC_ERR_TOO_LARGE;
    int64_t total = 0;
    for (int64_t c : cost) total += c;
    b->xbeg.assign(9, (int32_t)nit);
    b->xbeg[0] = 0;
    int64_t prefix = 0;
    int x = 1;
    for (int64_t i = 0; i < nit && x < 8; ++i) {
        while (x < 8 && prefix * 8 >= (int64_t)x * total) b->xbeg[x++] = (int32_t)i;
        prefix += cost[i];
    }
    for (int32_t m = 0; m < nmat; ++m) {
        const csrc_plan *p = b->plans[m];
        b->blob_off.push_back((int64_t)b->blob.size());
        b->blob.insert(b->blob.end(), p->blob.begin(), p->blob.end());
        b->blob.resize(csrc::align256((int64_t)b->blob.size()));
    }
    put_ints(b, b->items, b->off_items);
    put_ints(b, b->mitems, b->off_mitems);
    put_ints(b, b->xbeg, b->off_xbeg);
    b->off_descs = (int64_t)b->blob.size();
    b->off_parts = csrc::align256(b->off_descs + (int64_t)sizeof(csrc::MatDev) * std::max(1, nmat));
    b->ws_bytes = b->off_parts;
    return CSRC_OK;
}

}  // namespace

extern "C" int csrc_batch_plan_create(int32_t nmat, const int32_t *n, const int32_t *const *ia,
                                      const int32_t *const *ja, const int32_t *r, int32_t vdtype,
                                      const csrc_batch_opts *opts, csrc_batch_plan **out)
{
    if (!out || nmat < 0 || (nmat > 0 && (!n || !ia || !ja || !r))) return CSRC_ERR_ARG;
    if (vdtype < CSRC_F64 || vdtype > CSRC_BF16) return CSRC_ERR_ARG;
    *out = nullptr;
    csrc_batch_plan *b = nullptr;
    try {
        b = new csrc_batch_plan();
        b->nmat = nmat;
        b->vdtype = vdtype;
        if (opts) b->o = *opts;
        b->variant = b->o.variant == 0 ? CSRC_V_OWNER : b->o.variant;
        if (b->variant != CSRC_V_OWNER && b->variant != CSRC_V_PRIVATE) { delete b; return CSRC_ERR_ARG; }
        if (b->o.block == 0) b->o.block = b->variant == CSRC_V_OWNER ? 256 : 512;
        b->ydtype = vdtype == CSRC_F64 ? CSRC_F64 : (b->o.ydtype == CSRC_F64 ? CSRC_F64 : CSRC_F32);
        if (b->variant == CSRC_V_OWNER) {
            int st = owner_batch(b, nmat, n, ia, ja, r, vdtype);
            if (st) { delete b; return st; }
            *out = b;
            return CSRC_OK;
        }
        const int acc = csrc::acc_bytes(vdtype);
        const int C = csrc::mm_columns(vdtype);
        struct Item { int32_t m, t; int64_t cost; };
        std::vector<Item> work;
        int64_t part_bytes = 0;
        for (int32_t m = 0; m < nmat; ++m) {
            if (r[m] < 1 || r[m] > csrc::kMaxRhs || n[m] < 0) { delete b; return CSRC_ERR_ARG; }
            csrc_plan_opts po;
            csrc_plan_opts_default(CSRC_V_PRIVATE, &po);
            po.tile_work = b->o.tile_work;
            po.block = b->o.block;
            po.ydtype = b->ydtype;
            po.max_rhs = r[m];
            csrc_plan *p = nullptr;
            int st = csrc_plan_create(n[m], ia[m], ja[m], vdtype, &po, &p);
            if (st) { delete b; return st; }
            b->plans.push_back(p);
            b->n.push_back(n[m]);
            b->r.push_back(r[m]);
            b->smax = std::max(b->smax, p->max_span);
            b->emax = std::max(b->emax, p->max_tile_entries);
            b->ivmax = std::max(b->ivmax, p->max_intervals);
            b->part_off.push_back(part_bytes);
            part_bytes += csrc::align256(p->window_slots * r[m] * acc);
            const int chunks = (r[m] + C - 1) / C;
            for (int32_t t = 0; t < p->ntiles; ++t) {
                const int64_t e = (int64_t)p->tile_k[t + 1] - p->tile_k[t];
                const int64_t rows = (int64_t)p->tiles[t + 1] - p->tiles[t];
                work.push_back({m, t, (2 * e + rows) * chunks});
            }
            for (int32_t mb = 0; mb < p->nmerge_blocks; ++mb)
                if (p->mb_ptr[mb + 1] > p->mb_ptr[mb]) {
                    b->mitems.push_back(m);
                    b->mitems.push_back(mb);
                }
        }
        b->lds = csrc::lds_private_mm(b->smax, b->emax, b->ivmax, acc, C);
        if (b->lds > csrc::kLdsBudget) { delete b; return CSRC_ERR_UNSUPPORTED; }
        // longest items first, so the grid stride ends with short items
        std::stable_sort(work.begin(), work.end(), [](const Item &x, const Item &y) { return x.cost > y.cost; });
        for (const Item &w : work) {
            b->items.push_back(w.m);
            b->items.push_back(w.t);
        }
        // workspace image: per-matrix tables, then the two work lists
        for (int32_t m = 0; m < nmat; ++m) {
            const csrc_plan *p = b->plans[m];
            b->blob_off.push_back((int64_t)b->blob.size());
            b->blob.insert(b->blob.end(), p->blob.begin(), p->blob.end());
            b->blob.resize(csrc::align256((int64_t)b->blob.size()));
        }
        put_ints(b, b->items, b->off_items);
        put_ints(b, b->mitems, b->off_mitems);
        b->off_descs = (int64_t)b->blob.size();
        b->off_parts = csrc::align256(b->off_descs + (int64_t)sizeof(csrc::MatDev) * std::max(1, nmat));
        b->ws_bytes = csrc::align256(b->off_parts + part_bytes);
        *out = b;
        return CSRC_OK;
    } catch (const std::bad_alloc &) {
        delete b;
        return CSRC_ERR_NOMEM;
    }
}

extern "C" int csrc_batch_plan_destroy(csrc_batch_plan *b)
{
    delete b;
    return CSRC_OK;
}

extern "C" int64_t csrc_batch_workspace_bytes(const csrc_batch_plan *b) { return b ? b->ws_bytes : -1; }

extern "C" int csrc_batch_bind(const csrc_batch_plan *b, const csrc_matrix *A, const void *const *X,
                               const int64_t *ldx, void *const *Y, const int64_t *ldy, void *workspace,
                               int64_t ws_bytes, void *stream)
{
    if (!b || (b->nmat > 0 && (!A || !X || !ldx || !Y || !ldy))) return CSRC_ERR_ARG;
    if (!workspace || ws_bytes < b->ws_bytes) return CSRC_ERR_WORKSPACE;
    try {
        char *ws = static_cast<char *>(workspace);
        std::vector<csrc::MatDev> d(b->nmat);
        for (int32_t m = 0; m < b->nmat; ++m) {
            const csrc_plan *p = b->plans[m];
            const csrc_matrix &a = A[m];
            if (a.n != p->n || a.k != p->k || a.vdtype != b->vdtype) return CSRC_ERR_PLAN;
            if (ldx[m] < b->r[m] || ldy[m] < b->r[m]) return CSRC_ERR_ARG;
            if (a.n > 0 && (!X[m] || !Y[m] || !a.ia || !a.ad || (a.k > 0 && (!a.ja || !a.al || !a.au))))
                return CSRC_ERR_ARG;
            csrc::MatDev &md = d[m];
            md.P = csrc::plan_dev_at(p, ws + b->blob_off[m], ws + b->off_parts + b->part_off[m]);
            md.k = a.k;
            md.ia = a.ia;
            md.ja = a.ja;
            md.ad = a.ad;
            md.al = a.al;
            md.au = a.au;
            md.X = X[m];
            md.ldx = ldx[m];
            md.Y = Y[m];
            md.ldy = ldy[m];
            md.n = a.n;
            md.r = b->r[m];
            md.g = b->variant == CSRC_V_OWNER ? p->mm_group : 0;
            md.pad = 0;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        int st = csrc::hip_status(hipMemcpyAsync(ws, b->blob.data(), b->blob.size(), hipMemcpyHostToDevice, s));
        if (st) return st;
        if (b->nmat) {
            st = csrc::hip_status(hipMemcpyAsync(ws + b->off_descs, d.data(), sizeof(csrc::MatDev) * d.size(),
                                                 hipMemcpyHostToDevice, s));
            if (st) return st;
        }
        return csrc::hip_status(hipStreamSynchronize(s));
    } catch (const std::bad_alloc &) {
        return CSRC_ERR_NOMEM;
    }
}

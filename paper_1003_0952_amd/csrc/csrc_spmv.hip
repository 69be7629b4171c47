// CSRC products y = A x and y = A^T x on gfx950.
//
// Every variant evaluates, for each row i (Fig. 2a),
//     t_i = ad_i x_i + sum_{q in row i} al_q x_{ja_q}      (row-wise gather)
//     y_{ja_q} += au_q x_i  for each q in row i           (column-wise scatter)
// and differs only in how concurrent writes to y are resolved (Sec. 3).  The
// transpose product exchanges al and au (Sec. 5).
//
// Rows are processed by lane groups of G lanes (a "row segment"): the group
// streams its row's ja/al/au with consecutive lanes on consecutive entries,
// so a wave reads 64/G consecutive rows as one contiguous span; the row sum
// is reduced with lane shuffles.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "device_common.h"
#include "internal.h"

namespace csrc {

constexpr int kUnroll = 4;   // row groups in flight per lane group

// Walks rows row_at(idx) for idx in [ib, ie) step ngrp (this group: grp).
//   ia_at(r), xr_at(r), d_at(r): row bounds, x_r and ad_r
//   entry(j, a, w): returns a * x_j and scatters w = au * x_r to y_j
//   done(r, t):     commits the finished row value t = ad_r x_r + sum
template <int G, class V, class A, class RowAt, class IaAt, class XrAt, class DAt, class Entry,
          class Done>
__device__ __forceinline__ void rows_loop(int ib, int ie, int grp, int ngrp, int lg, RowAt row_at,
                                          IaAt ia_at, XrAt xr_at, DAt d_at,
                                          const int32_t *__restrict__ ja,
                                          const V *__restrict__ al, const V *__restrict__ au,
                                          Entry entry, Done done)
{
    for (int base = ib + grp; base < ie; base += kUnroll * ngrp) {
        int r[kUnroll], q0[kUnroll], q1[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int idx = base + u * ngrp;
            bool ok = idx < ie;
            r[u] = ok ? row_at(idx) : -1;
            q0[u] = ok ? ia_at(r[u]) : 0;
            q1[u] = ok ? ia_at(r[u] + 1) : 0;
        }
        int j[kUnroll];
        A a[kUnroll], b[kUnroll], xr[kUnroll], d[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            int q = q0[u] + lg;
            bool ok = q < q1[u];
            j[u] = ok ? ja[q] : 0;
            a[u] = ok ? (A)ldv(al, q) : A(0);
            b[u] = ok ? (A)ldv(au, q) : A(0);
            bool rv = r[u] >= 0;
            xr[u] = rv ? xr_at(r[u]) : A(0);
            d[u] = rv ? d_at(r[u]) : A(0);
        }
        A acc[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            acc[u] = A(0);
            if (q0[u] + lg < q1[u]) acc[u] = entry(j[u], a[u], b[u] * xr[u]);
            for (int q = q0[u] + lg + G; q < q1[u]; q += G)
                acc[u] += entry(ja[q], (A)ldv(al, q), (A)ldv(au, q) * xr[u]);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            A s = group_sum<G>(acc[u]);
            if (lg == 0 && r[u] >= 0) done(r[u], d[u] * xr[u] + s);
        }
    }
}

// ---------------------------------------------------------------- helpers

template <class YT>
__global__ void k_fill_zero(YT *__restrict__ y, int32_t n, int32_t r, int64_t ldy)
{
    int64_t total = (int64_t)n * r;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t i = e / r, c = e - i * r;
        y[i * ldy + c] = YT(0);
    }
}

// last index i in [0, cnt) with key[i] <= v (key ascending, key[0] <= v)
__device__ __forceinline__ int upper_index(const int32_t *key, int cnt, int v)
{
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (key[mid] <= v) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ PLAIN

// One thread per row, y cleared beforehand, global atomics for everything.
template <class VT, class YT>
__global__ __launch_bounds__(256) void k_plain(int32_t n, const int32_t *__restrict__ ia,
                                               const int32_t *__restrict__ ja,
                                               const typename VT::V *__restrict__ ad,
                                               const typename VT::V *__restrict__ al,
                                               const typename VT::V *__restrict__ au,
                                               const typename VT::X *__restrict__ x,
                                               YT *__restrict__ y)
{
    using A = typename VT::A;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    A xi = (A)x[i];
    A t = (A)ldv(ad, i) * xi;
    for (int q = ia[i]; q < ia[i + 1]; ++q) {
        int j = ja[q];
        t += (A)ldv(al, q) * (A)x[j];
        atomic_add(&y[j], (YT)((A)ldv(au, q) * xi));
    }
    atomic_add(&y[i], (YT)t);
}

// ----------------------------------------------------------------- ATOMIC

template <int G, class VT, class YT>
__global__ __launch_bounds__(512) void k_atomic(const int32_t *__restrict__ tiles,
                                                const int32_t *__restrict__ ia,
                                                const int32_t *__restrict__ ja,
                                                const typename VT::V *__restrict__ ad,
                                                const typename VT::V *__restrict__ al,
                                                const typename VT::V *__restrict__ au,
                                                const typename VT::X *__restrict__ x,
                                                YT *__restrict__ y)
{
    using A = typename VT::A;
    int t = xcd_tile(blockIdx.x, gridDim.x);
    int r0 = tiles[t], r1 = tiles[t + 1];
    int lg = threadIdx.x % G, grp = threadIdx.x / G, ngrp = blockDim.x / G;
    rows_loop<G, typename VT::V, A>(
        r0, r1, grp, ngrp, lg, [](int i) { return i; }, [&](int r) { return ia[r]; },
        [&](int r) { return (A)x[r]; }, [&](int r) { return (A)ldv(ad, r); }, ja, al, au,
        [&](int j, A a, A w) -> A {
            atomic_add(&y[j], (YT)w);
            return a * (A)x[j];
        },
        [&](int r, A v) { atomic_add(&y[r], (YT)v); });
}

// ---------------------------------------------------------------- PRIVATE

// Local buffers of Sec. 3.1 kept in LDS: a tile of rows [r0, r1) accumulates
// its own rows (s_y) and its effective range below r0 (s_w, compact window
// slots).  x of both ranges is staged in LDS first (s_x, s_xw).  Own rows go
// to y; window slots go to the partial buffer for the merge pass.
template <int G, class VT, class YT>
__global__ __launch_bounds__(512) void k_private(PlanDev P, const int32_t *__restrict__ ia,
                                                 const int32_t *__restrict__ ja,
                                                 const typename VT::V *__restrict__ ad,
                                                 const typename VT::V *__restrict__ al,
                                                 const typename VT::V *__restrict__ au,
                                                 const typename VT::X *__restrict__ x,
                                                 YT *__restrict__ y, int tmax, int wmax, int ivmax)
{
    using A = typename VT::A;
    extern __shared__ __align__(16) unsigned char lds[];
    A *s_x = reinterpret_cast<A *>(lds);
    A *s_y = s_x + tmax;
    A *s_xw = s_y + tmax;
    A *s_w = s_xw + wmax;
    int32_t *s_ia = reinterpret_cast<int32_t *>(s_w + wmax);
    int32_t *s_ivrow = s_ia + tmax + 1;
    int32_t *s_ivslot = s_ivrow + ivmax;

    const int tid = threadIdx.x, B = blockDim.x;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r0 = P.tiles[t], r1 = P.tiles[t + 1], T = r1 - r0;
    const int e0 = P.iv_ptr[t], NI = P.iv_ptr[t + 1] - e0;
    const int W = NI ? P.iv_slot[e0 + NI - 1] + P.iv_len[e0 + NI - 1] : 0;

    for (int i = tid; i < T; i += B) {
        s_ia[i] = ia[r0 + i];
        s_x[i] = (A)x[r0 + i];
        s_y[i] = A(0);
    }
    if (tid == 0) s_ia[T] = ia[r1];
    for (int i = tid; i < NI; i += B) {
        s_ivrow[i] = P.iv_row[e0 + i];
        s_ivslot[i] = P.iv_slot[e0 + i];
    }
    __syncthreads();
    for (int s = tid; s < W; s += B) {
        int k = upper_index(s_ivslot, NI, s);
        s_xw[s] = (A)x[s_ivrow[k] + (s - s_ivslot[k])];
        s_w[s] = A(0);
    }
    __syncthreads();

    const int lg = tid % G, grp = tid / G, ngrp = B / G;
    rows_loop<G, typename VT::V, A>(
        r0, r1, grp, ngrp, lg, [](int i) { return i; }, [&](int r) { return s_ia[r - r0]; },
        [&](int r) { return s_x[r - r0]; }, [&](int r) { return (A)ldv(ad, r); }, ja, al, au,
        [&](int j, A a, A w) -> A {
            if (j >= r0) {
                atomic_add(&s_y[j - r0], w);
                return a * s_x[j - r0];
            }
            int k = upper_index(s_ivrow, NI, j);
            int sl = s_ivslot[k] + (j - s_ivrow[k]);
            atomic_add(&s_w[sl], w);
            return a * s_xw[sl];
        },
        [&](int r, A v) { atomic_add(&s_y[r - r0], v); });
    __syncthreads();

    for (int i = tid; i < T; i += B) y[r0 + i] = (YT)s_y[i];
    if (W) {
        A *part = reinterpret_cast<A *>(P.partials) + P.iv_goff[e0];
        for (int s = tid; s < W; s += B) part[s] = s_w[s];
    }
}

// Merge pass: y_i += partial slots covering i, in ascending tile order.
// MT is the merge type; COMP adds a TwoSum (Knuth) error term.
template <class A, class YT, class MT, bool COMP>
__global__ __launch_bounds__(kMergeBlock) void k_merge(int32_t n, PlanDev P, YT *__restrict__ y)
{
    const int b = blockIdx.x;
    const int e0 = P.mb_ptr[b], e1 = P.mb_ptr[b + 1];
    const int i = b * kMergeBlock + threadIdx.x;
    if (e0 == e1 || i >= n) return;
    const A *part = reinterpret_cast<const A *>(P.partials);
    MT s = (MT)y[i], c = MT(0);
    for (int e = e0; e < e1; ++e) {
        int g = P.mb_iv[e];
        int a = P.iv_row[g], L = P.iv_len[g];
        if (i >= a && i < a + L) {
            MT v = (MT)part[P.iv_goff[g] + (i - a)];
            if (COMP) {
                MT s2 = s + v;
                MT bp = s2 - s;
                c += (s - (s2 - bp)) + (v - bp);
                s = s2;
            } else {
                s += v;
            }
        }
    }
    y[i] = (YT)(s + c);
}

// ------------------------------------------------------------------ OWNER

// Owner computes: the tile's own rows gather (out-of-tile x from L2) and
// scatter only into the tile; then the tile visits the rows of later tiles
// that scatter into it (pull intervals) and adds those contributions.  Each
// y entry is completed in one workgroup's LDS and stored once.
template <int G, class VT, class YT>
__global__ __launch_bounds__(512) void k_owner(PlanDev P, const int32_t *__restrict__ ia,
                                               const int32_t *__restrict__ ja,
                                               const typename VT::V *__restrict__ ad,
                                               const typename VT::V *__restrict__ al,
                                               const typename VT::V *__restrict__ au,
                                               const typename VT::X *__restrict__ x,
                                               YT *__restrict__ y, int tmax)
{
    using A = typename VT::A;
    using V = typename VT::V;
    extern __shared__ __align__(16) unsigned char lds[];
    A *s_x = reinterpret_cast<A *>(lds);
    A *s_y = s_x + tmax;
    int32_t *s_ia = reinterpret_cast<int32_t *>(s_y + tmax);

    const int tid = threadIdx.x, B = blockDim.x;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r0 = P.tiles[t], r1 = P.tiles[t + 1], T = r1 - r0;
    for (int i = tid; i < T; i += B) {
        s_ia[i] = ia[r0 + i];
        s_x[i] = (A)x[r0 + i];
        s_y[i] = A(0);
    }
    if (tid == 0) s_ia[T] = ia[r1];
    __syncthreads();

    const int lg = tid % G, grp = tid / G, ngrp = B / G;
    rows_loop<G, V, A>(
        r0, r1, grp, ngrp, lg, [](int i) { return i; }, [&](int r) { return s_ia[r - r0]; },
        [&](int r) { return s_x[r - r0]; }, [&](int r) { return (A)ldv(ad, r); }, ja, al, au,
        [&](int j, A a, A w) -> A {
            if (j >= r0) {
                atomic_add(&s_y[j - r0], w);
                return a * s_x[j - r0];
            }
            return a * (A)x[j];
        },
        [&](int r, A v) { atomic_add(&s_y[r - r0], v); });

    // pulled rows: only their entries with targets inside [r0, r1)
    const int p0 = P.iv_ptr[t], p1 = P.iv_ptr[t + 1];
    for (int e = p0; e < p1; ++e) {
        const int a0 = P.iv_row[e], L = P.iv_len[e];
        for (int base = grp; base < L; base += kUnroll * ngrp) {
            int q0[kUnroll], q1[kUnroll];
            A xi[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                int idx = base + u * ngrp;
                bool ok = idx < L;
                int r = a0 + idx;
                q0[u] = ok ? ia[r] : 0;
                q1[u] = ok ? ia[r + 1] : 0;
                xi[u] = ok ? (A)x[r] : A(0);
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                for (int q = q0[u] + lg; q < q1[u]; q += G) {
                    int j = ja[q];
                    if (j >= r0 && j < r1) atomic_add(&s_y[j - r0], (A)ldv(au, q) * xi[u]);
                }
            }
        }
    }
    __syncthreads();
    for (int i = tid; i < T; i += B) y[r0 + i] = (YT)s_y[i];
}

// ------------------------------------------------------------------ COLOR

// One colour class [c0, c1) of the row list: write sets of its rows are
// pairwise disjoint (Sec. 3.2), so y is updated with plain loads and stores.
template <int G, class VT, class YT>
__global__ __launch_bounds__(512) void k_color(const int32_t *__restrict__ crow, int c0, int c1,
                                               const int32_t *__restrict__ ia,
                                               const int32_t *__restrict__ ja,
                                               const typename VT::V *__restrict__ ad,
                                               const typename VT::V *__restrict__ al,
                                               const typename VT::V *__restrict__ au,
                                               const typename VT::X *__restrict__ x,
                                               YT *__restrict__ y)
{
    using A = typename VT::A;
    const int lg = threadIdx.x % G;
    const int grp = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
    const int ngrp = gridDim.x * (blockDim.x / G);
    rows_loop<G, typename VT::V, A>(
        c0, c1, grp, ngrp, lg, [&](int idx) { return crow[idx]; }, [&](int r) { return ia[r]; },
        [&](int r) { return (A)x[r]; }, [&](int r) { return (A)ldv(ad, r); }, ja, al, au,
        [&](int j, A a, A w) -> A {
            y[j] = y[j] + (YT)w;
            return a * (A)x[j];
        },
        [&](int r, A v) { y[r] = y[r] + (YT)v; });
}

// --------------------------------------------------------------- dispatch

static PlanDev plan_dev(const csrc_plan *p, void *ws)
{
    char *b = static_cast<char *>(ws);
    auto at = [&](const Table &t) -> const void * { return b ? b + t.offset : nullptr; };
    PlanDev d;
    d.tiles = (const int32_t *)at(p->t_tiles);
    d.iv_ptr = (const int32_t *)at(p->t_iv_ptr);
    d.iv_row = (const int32_t *)at(p->t_iv_row);
    d.iv_len = (const int32_t *)at(p->t_iv_len);
    d.iv_slot = (const int32_t *)at(p->t_iv_slot);
    d.iv_goff = (const int64_t *)at(p->t_iv_goff);
    d.mb_ptr = (const int32_t *)at(p->t_mb_ptr);
    d.mb_iv = (const int32_t *)at(p->t_mb_iv);
    d.crow = (const int32_t *)at(p->t_crow);
    d.cptr = nullptr;
    d.partials = b ? b + p->t_partials.offset : nullptr;
    return d;
}

static int fill_grid(int64_t count) { return (int)std::min<int64_t>(4096, std::max<int64_t>(1, (count + 255) / 256)); }

template <class VT, class YT, int G>
static int launch_variant(const csrc_plan *p, const csrc_matrix *A, const void *al_, const void *au_,
                          const void *x_, void *y_, void *ws, hipStream_t s)
{
    using V = typename VT::V;
    using X = typename VT::X;
    using Acc = typename VT::A;
    const int32_t n = A->n;
    const V *ad = static_cast<const V *>(A->ad);
    const V *al = static_cast<const V *>(al_);
    const V *au = static_cast<const V *>(au_);
    const X *x = static_cast<const X *>(x_);
    YT *y = static_cast<YT *>(y_);
    const int B = p->o.block;
    PlanDev P = plan_dev(p, ws);
    switch (p->o.variant) {
    case CSRC_V_PLAIN:
        k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
        k_plain<VT, YT><<<(n + 255) / 256, 256, 0, s>>>(n, A->ia, A->ja, ad, al, au, x, y);
        break;
    case CSRC_V_ATOMIC:
        k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
        k_atomic<G, VT, YT><<<p->ntiles, B, 0, s>>>(P.tiles, A->ia, A->ja, ad, al, au, x, y);
        break;
    case CSRC_V_PRIVATE: {
        int tmax = p->max_tile_rows, wmax = p->max_window, ivmax = p->max_intervals;
        size_t lds = (size_t)(2 * tmax + 2 * wmax) * sizeof(Acc) + (size_t)(tmax + 1 + 2 * ivmax + 1) * 4;
        auto kern = k_private<G, VT, YT>;
        if (lds > 65536)
            hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        kern<<<p->ntiles, B, lds, s>>>(P, A->ia, A->ja, ad, al, au, x, y, tmax, wmax, ivmax);
        if (p->nmerge_blocks > 0 && p->window_slots > 0) {
            if (std::is_same<YT, double>::value)
                k_merge<Acc, YT, double, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
            else if (p->o.compensated)
                k_merge<Acc, YT, float, true><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
            else
                k_merge<Acc, YT, float, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
        }
        break;
    }
    case CSRC_V_OWNER: {
        int tmax = p->max_tile_rows;
        size_t lds = (size_t)(2 * tmax) * sizeof(Acc) + (size_t)(tmax + 1) * 4;
        auto kern = k_owner<G, VT, YT>;
        if (lds > 65536)
            hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        kern<<<p->ntiles, B, lds, s>>>(P, A->ia, A->ja, ad, al, au, x, y, tmax);
        break;
    }
    case CSRC_V_COLOR: {
        k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
        for (int c = 0; c < p->ncolors; ++c) {
            int c0 = p->cptr[c], c1 = p->cptr[c + 1];
            int rows_per_block = (B / G) * kUnroll;
            int grid = std::max(1, std::min(65535, (c1 - c0 + rows_per_block - 1) / rows_per_block));
            k_color<G, VT, YT><<<grid, B, 0, s>>>(P.crow, c0, c1, A->ia, A->ja, ad, al, au, x, y);
        }
        break;
    }
    default:
        return CSRC_ERR_ARG;
    }
    return hipGetLastError() == hipSuccess ? CSRC_OK : CSRC_ERR_HIP;
}

template <class VT, class YT>
static int launch_lanes(const csrc_plan *p, const csrc_matrix *A, const void *al, const void *au,
                        const void *x, void *y, void *ws, hipStream_t s)
{
    switch (p->o.lanes) {
    case 2: return launch_variant<VT, YT, 2>(p, A, al, au, x, y, ws, s);
    case 4: return launch_variant<VT, YT, 4>(p, A, al, au, x, y, ws, s);
    case 8: return launch_variant<VT, YT, 8>(p, A, al, au, x, y, ws, s);
    case 16: return launch_variant<VT, YT, 16>(p, A, al, au, x, y, ws, s);
    case 32: return launch_variant<VT, YT, 32>(p, A, al, au, x, y, ws, s);
    case 64: return launch_variant<VT, YT, 64>(p, A, al, au, x, y, ws, s);
    default: return CSRC_ERR_PLAN;
    }
}

static int xbytes(int32_t vd) { return vd == CSRC_F64 ? 8 : 4; }

static bool overlap(const void *a, int64_t an, const void *b, int64_t bn)
{
    const char *pa = static_cast<const char *>(a), *pb = static_cast<const char *>(b);
    return pa < pb + bn && pb < pa + an;
}

int check_call(const csrc_matrix *A, const csrc_plan *p, void *ws, int64_t ws_bytes)
{
    if (!A || !p) return CSRC_ERR_ARG;
    if (A->n < 0 || A->k < 0) return CSRC_ERR_ARG;
    if (A->n != p->n || A->k != p->k || A->vdtype != p->vdtype) return CSRC_ERR_PLAN;
    if (A->n > 0 && (!A->ia || !A->ad || (A->k > 0 && (!A->ja || !A->al || !A->au)))) return CSRC_ERR_ARG;
    if (p->ws_bytes > 0 && (!ws || ws_bytes < p->ws_bytes)) return CSRC_ERR_WORKSPACE;
    return CSRC_OK;
}

static int product(const csrc_matrix *A, const csrc_plan *p, const void *x, void *y, void *ws,
                   int64_t ws_bytes, void *stream, bool transpose)
{
    int st = check_call(A, p, ws, ws_bytes);
    if (st) return st;
    if (A->n == 0) return CSRC_OK;
    if (!x || !y) return CSRC_ERR_ARG;
    int ys = (A->vdtype == CSRC_F64 || p->o.ydtype == CSRC_F64) ? 8 : 4;
    if (overlap(x, (int64_t)A->n * xbytes(A->vdtype), y, (int64_t)A->n * ys)) return CSRC_ERR_ALIAS;
    const void *al = transpose ? A->au : A->al;
    const void *au = transpose ? A->al : A->au;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (A->vdtype) {
    case CSRC_F64: return launch_lanes<F64T, double>(p, A, al, au, x, y, ws, s);
    case CSRC_F32:
        return p->o.ydtype == CSRC_F64 ? launch_lanes<F32T, double>(p, A, al, au, x, y, ws, s)
                                       : launch_lanes<F32T, float>(p, A, al, au, x, y, ws, s);
    case CSRC_BF16:
        return p->o.ydtype == CSRC_F64 ? launch_lanes<B16T, double>(p, A, al, au, x, y, ws, s)
                                       : launch_lanes<B16T, float>(p, A, al, au, x, y, ws, s);
    default: return CSRC_ERR_ARG;
    }
}

}  // namespace csrc

extern "C" int csrc_spmv(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y,
                         void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, x, y, workspace, ws_bytes, stream, false);
}

extern "C" int csrc_spmv_t(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y,
                           void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, x, y, workspace, ws_bytes, stream, true);
}

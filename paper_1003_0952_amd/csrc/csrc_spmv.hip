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
#include <mutex>
#include <type_traits>

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

// y[i * ldy + c] = 0 for rows i < n, columns c < r.  A contiguous block
// (ldy == r) is cleared with 16-byte stores after a short unaligned head.
template <class YT>
__global__ __launch_bounds__(256) void k_fill_zero(YT *__restrict__ y, int32_t n, int32_t r, int64_t ldy)
{
    const int64_t gt = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t gs = (int64_t)gridDim.x * blockDim.x;
    if (ldy == r) {
        constexpr int V = 16 / sizeof(YT);
        const int64_t count = (int64_t)n * r;
        const int64_t mis = (int64_t)((reinterpret_cast<uintptr_t>(y) & 15) / sizeof(YT));
        const int64_t head = mis ? min<int64_t>(count, V - mis) : 0;
        if (gt < head) y[gt] = YT(0);
        int4 *b = reinterpret_cast<int4 *>(y + head);
        const int64_t nv = (count - head) / V;
        // one contiguous run of 16-byte words per workgroup (HBM row locality)
        const int64_t per = (nv + gridDim.x - 1) / gridDim.x;
        const int64_t v0 = blockIdx.x * per, v1 = min(nv, v0 + per);
        for (int64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) b[v] = make_int4(0, 0, 0, 0);
        const int64_t t0 = head + nv * V;
        if (t0 + gt < count) y[t0 + gt] = YT(0);
        return;
    }
    for (int64_t i = gt; i < n; i += gs)
        for (int c = 0; c < r; ++c) y[i * ldy + c] = YT(0);
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
                                               const typename VT::X *__restrict__ x, int64_t ldx,
                                               YT *__restrict__ y, int64_t ldy)
{
    using A = typename VT::A;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    A xi = (A)x[i * ldx];
    A t = (A)ldv(ad, i) * xi;
    for (int q = ia[i]; q < ia[i + 1]; ++q) {
        int j = ja[q];
        t += (A)ldv(al, q) * (A)x[j * ldx];
        atomic_add(&y[j * ldy], (YT)((A)ldv(au, q) * xi));
    }
    atomic_add(&y[i * ldy], (YT)t);
}

// ------------------------------------------------------- flat tile engine
//
// The tile kernels stream the stored entries of a row block [r0, r1), i.e.
// entries [k0, k1) = [ia[r0], ia[r1]).  A batch covers 4B consecutive
// entries (B = workgroup size); lane l owns the pairs at 2l and 2B + 2l, so
// every load instruction (ja as 8 bytes, al and au as 2 values) reads one
// contiguous span across the wave.  Loads are non-temporal where the data is
// read once.  The stream is software pipelined: the next batch's loads are
// in flight while the current batch is processed.  The row of each entry
// comes from an LDS table of uint16 row ids (relative to the block) filled
// from ia; a lane's partial row sums are flushed into LDS when the row
// changes.

typedef int i2v __attribute__((ext_vector_type(2)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));

constexpr uint32_t kNoRow = 0xFFFF;

// Buffer descriptor over n bytes at p (raw addressing, stride 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, (int)bytes, 0x00020000);
}

// The stored entries [kb, ke) of ja, al and au (kb even) behind buffer
// descriptors.  Raw buffer loads check every dword against the descriptor
// size: a dword at or past entry ke reads as zero and touches no memory.  So
// a pair load at an even q needs no tail branch (a branch whose else-path
// loads makes the compiler drain every outstanding load before the next
// one), never reads past the range, and entries past ke come back as zero.
// NT marks data read once (non-temporal).
template <class VT, bool NT>
struct Entries {
    using V = typename VT::V;
    using A = typename VT::A;
    static constexpr int kAux = NT ? 2 : 0;
    __amdgpu_buffer_rsrc_t rj, ra, ru;
    int kb, ke;

    // pad: the value ranges end on a 4-byte boundary, i.e. a bfloat16 pair
    // that straddles ke is read whole (its second value, entry ke, is not
    // this range's and is ignored by the caller).  Only for ranges whose
    // entry ke exists in the arrays.
    __device__ __forceinline__ Entries(const int32_t *ja, const V *al, const V *au, int kb_, int ke_,
                                       bool pad = false)
        : kb(kb_), ke(ke_)
    {
        const uint32_t n = (uint32_t)max(ke_ - kb_, 0);
        const uint32_t vb = n * (uint32_t)sizeof(V);
        rj = make_rsrc(ja + kb_, n * 4u);
        ra = make_rsrc(al + kb_, pad ? (vb + 3u) & ~3u : vb);
        ru = make_rsrc(au + kb_, pad ? (vb + 3u) & ~3u : vb);
    }

    // the two bfloat16 values of the pair at q as one raw word (low half:
    // entry q); a word past the range reads as zero
    __device__ __forceinline__ uint32_t w2(__amdgpu_buffer_rsrc_t r, int q) const
    {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (q - kb) * 2, 0, kAux);
    }

    __device__ __forceinline__ void j2(int q, int (&o)[2]) const
    {
        const i2v v = __builtin_bit_cast(i2v, __builtin_amdgcn_raw_buffer_load_b64(rj, (q - kb) * 4, 0, kAux));
        o[0] = v.x;
        o[1] = v.y;
    }
    __device__ __forceinline__ void v2(__amdgpu_buffer_rsrc_t r, int q, double (&o)[2]) const
    {
        const d2v v = __builtin_bit_cast(d2v, __builtin_amdgcn_raw_buffer_load_b128(r, (q - kb) * 8, 0, kAux));
        o[0] = v.x;
        o[1] = v.y;
    }
    __device__ __forceinline__ void v2(__amdgpu_buffer_rsrc_t r, int q, float (&o)[2]) const
    {
        if constexpr (std::is_same<V, float>::value) {
            const f2v v = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, (q - kb) * 4, 0, kAux));
            o[0] = v.x;
            o[1] = v.y;
        } else {
            // bfloat16: one dword holds the pair; a dword that ends past the
            // range reads as zero, so the lane whose pair straddles ke takes
            // its first element from a 2-byte load (other lanes pass an
            // offset outside the range: no memory access).
            const int off = (q - kb) * 2;
            const bool straddle = q + 1 == ke;
            const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kAux);
            const uint16_t h = __builtin_amdgcn_raw_buffer_load_b16(r, straddle ? off : 0x7FFFFFF0, 0, kAux);
            o[0] = __uint_as_float((straddle ? (uint32_t)h : (w & 0xFFFFu)) << 16);
            o[1] = __uint_as_float(w & 0xFFFF0000u);
        }
    }
    __device__ __forceinline__ void al2(int q, A (&o)[2]) const { v2(ra, q, o); }
    __device__ __forceinline__ void au2(int q, A (&o)[2]) const { v2(ru, q, o); }
};

// Fill s_rid[q - kb] = row - ra for the entries of rows [ra, rb), i.e.
// [ia[ra], ia[rb]), and kNoRow on [kb, ia[ra]) and on [ia[rb], round2(...) + 2)
// so every pair read of the stream finds a defined value.  kb is ia[ra]
// rounded down to even.
__device__ __forceinline__ void fill_row_ids(const int32_t *__restrict__ ia, int ra, int rb, int kb,
                                            uint16_t *s_rid)
{
    const int tid = threadIdx.x, B = blockDim.x;
    const int k0 = ia[ra], k1 = ia[rb];
    const int len = ((k1 - kb) + 3) & ~1;
    for (int s = tid; s < k0 - kb; s += B) s_rid[s] = kNoRow;
    for (int s = (k1 - kb) + tid; s < len; s += B) s_rid[s] = kNoRow;
    for (int i = tid; i < rb - ra; i += B) {
        const int q0 = ia[ra + i], q1 = ia[ra + i + 1];
        for (int q = q0; q < q1; ++q) s_rid[q - kb] = (uint16_t)i;
    }
}

// One lane's share of a batch: NP pairs at qb, qb + 2B, ... of the entries
// E (a batch covers 2 NP B consecutive entries).  LOAD_AL / LOAD_AU select
// which value arrays are fetched up front (the others read as zero).  Pairs
// past the range of E read as zero.
template <class VT, bool LOAD_AL, bool LOAD_AU, bool NT, int NP = 2>
struct Batch {
    using A = typename VT::A;
    using V = typename VT::V;
    static constexpr int kPairs = NP;
    int j[NP][2];
    A a[NP][2];
    A u[NP][2];

    __device__ __forceinline__ void load(int qb, const Entries<VT, NT> &E)
    {
        const int half = 2 * (int)blockDim.x;
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            const int q = qb + half * s;
            E.j2(q, j[s]);
            if (LOAD_AL) E.al2(q, a[s]);
            else a[s][0] = a[s][1] = A(0);
            if constexpr (VT::kSym) {
                static_assert(LOAD_AL && LOAD_AU, "symmetric storage loads al for both");
                u[s][0] = a[s][0];
                u[s][1] = a[s][1];
            } else if (LOAD_AU) {
                E.au2(q, u[s]);
            } else {
                u[s][0] = u[s][1] = A(0);
            }
        }
    }
};

// A lane's share of a batch for the branch-free stream (process_batch_flat):
// NP pairs at qb, qb + 2B, ... of E, every value array loaded.  bfloat16
// pairs stay raw words until they are used, so the load of the next batch is
// never waited for while the current one is processed (E must be padded).
template <class VT, bool NT, int NP>
struct PairBatch {
    using A = typename VT::A;
    static constexpr int kPairs = NP;
    static constexpr bool kRaw = std::is_same<typename VT::V, uint16_t>::value;
    int j[NP][2];
    A a[kRaw ? 1 : NP][2];
    A u[kRaw || VT::kSym ? 1 : NP][2];
    uint32_t aw[kRaw ? NP : 1], uw[kRaw && !VT::kSym ? NP : 1];

    __device__ __forceinline__ void load(int qb, const Entries<VT, NT> &E)
    {
        const int half = 2 * (int)blockDim.x;
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            const int q = qb + half * s;
            E.j2(q, j[s]);
            if constexpr (kRaw) {
                aw[s] = E.w2(E.ra, q);
                if constexpr (!VT::kSym) uw[s] = E.w2(E.ru, q);
            } else {
                E.al2(q, a[s]);
                if constexpr (!VT::kSym) E.au2(q, u[s]);
            }
        }
    }
    __device__ __forceinline__ A al(int s, int e) const
    {
        if constexpr (kRaw) return __uint_as_float(e ? aw[s] & 0xFFFF0000u : aw[s] << 16);
        else return a[s][e];
    }
    __device__ __forceinline__ A au(int s, int e) const
    {
        if constexpr (VT::kSym) return al(s, e);
        else if constexpr (kRaw) return __uint_as_float(e ? uw[s] & 0xFFFF0000u : uw[s] << 16);
        else return u[s][e];
    }
};

struct NoHook {
    __device__ __forceinline__ void operator()() const {}
};

// Wait for every outstanding memory operation.  Placed where everything has
// landed anyway (after staging), it resets the compiler's per-register
// pending-load state, which it otherwise merges conservatively over the
// staging code's divergent paths and turns into waits on the next batch
// inside the stream loop.
__device__ __forceinline__ void settle_loads() { __builtin_amdgcn_s_waitcnt(0); }

// Lane exchange inside groups of 4 and 8 lanes (DPP: quad permutation and
// half-row mirror), for 32- and 64-bit values.  Every lane of the wave must
// be active.
template <int CTRL>
__device__ __forceinline__ int dpp(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v)
{
    return __int_as_float(dpp<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v)
{
    const i2v p = __builtin_bit_cast(i2v, v);
    i2v q;
    q.x = dpp<CTRL>(p.x);
    q.y = dpp<CTRL>(p.y);
    return __builtin_bit_cast(double, q);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <-> 7 - i within each group of 8
constexpr int kDppQuadFirst = 0x00;   // quad_perm [0,0,0,0]
constexpr int kDppQuadLast = 0xFF;    // quad_perm [3,3,3,3]

// Flush a lane's pair of gathered products (rows r0 <= r1 of its two
// entries, kNoRow for none).  Consecutive lanes often hold pairs of one long
// row, and their LDS adds to one address are serialised; so the pair sums of
// a row segment are first reduced across lanes: when all 8 (else all 4)
// lanes of an aligned group hold one pair of the same row, the group's first
// lane adds the group's total.  Called by every lane of the wave.
template <class A, class Flush>
__device__ __forceinline__ void flush_pairs(int r0, int r1, A g0, A g1, Flush flush)
{
    const int lane = (int)(threadIdx.x & 63);
    const bool one = r0 == r1 && r0 != (int)kNoRow;
    const int key = one ? r0 : -1 - lane;          // distinct for lanes that do not take part
    const A v = g0 + g1;
    // every exchange is evaluated by all lanes before any branch (a lane
    // exchange under a partial exec mask reads undefined values): no
    // short-circuit operators here
    const int k1 = dpp<kDppXor1>(key), k2 = dpp<kDppXor2>(key);
    const int k3 = dpp<kDppXor1>(k2);
    const bool quad = (key == k1) & (key == k2) & (key == k3);
    A vq = v + dpp<kDppXor1>(v);
    vq = vq + dpp<kDppXor2>(vq);
    const int kq = quad ? key : -1 - (lane | 64);   // a quad's key when the whole quad is one row
    const int km = dpp<kDppHalfMirror>(kq);
    const bool oct = quad & (kq == km);
    const A vo = vq + dpp<kDppHalfMirror>(vq);
    if (oct) {
        if ((lane & 7) == 0) flush(r0, vo);
    } else if (quad) {
        if ((lane & 3) == 0) flush(r0, vq);
    } else if (one) {
        flush(r0, v);
    } else {
        if (r0 != (int)kNoRow) flush(r0, g0);
        if (r1 != (int)kNoRow) flush(r1, g1);
    }
}

// Process one batch held in cur (lane pairs at qb, qb + 2B, ... of the
// entries E): for each entry of row r (relative) with column j,
// x_j = ent(j, au * s_x[r]) scatters and gathers, and a lane's run of
// gathered products of one row goes to flush(r, sum).  With LOAD_AU false,
// an au pair is fetched only if need_au(j) holds for one of its entries
// (else its products are zero and ent ignores them).
template <class VT, bool LOAD_AU, bool NT, int NP, class NeedAu, class Ent, class Flush>
__device__ __forceinline__ void process_batch(Batch<VT, true, LOAD_AU, NT, NP> &cur, int qb,
                                              const Entries<VT, NT> &E, const uint16_t *__restrict__ s_rid,
                                              const typename VT::A *s_x, NeedAu need_au, Ent ent, Flush flush)
{
    using A = typename VT::A;
    const int half = 2 * (int)blockDim.x;
    const int kb = E.kb, k1 = E.ke;
    uint32_t rv[NP];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int q = qb + half * s;
        rv[s] = q < k1 ? *reinterpret_cast<const uint32_t *>(s_rid + (q - kb)) : 0xFFFFFFFFu;
    }
    if (!LOAD_AU) {
#pragma unroll
        for (int s = 0; s < NP; ++s) {
            const bool need = ((rv[s] & 0xFFFF) != kNoRow && need_au(cur.j[s][0])) ||
                              ((rv[s] >> 16) != kNoRow && need_au(cur.j[s][1]));
            if (need) E.au2(qb + half * s, cur.u[s]);
            else cur.u[s][0] = cur.u[s][1] = A(0);
        }
    }
    // x of the entries' own rows, read before any LDS update of the batch
    A xr[NP][2];
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int r0 = (int)(rv[s] & 0xFFFF), r1 = (int)(rv[s] >> 16);
        xr[s][0] = s_x[r0 != (int)kNoRow ? r0 : 0];
        xr[s][1] = s_x[r1 != (int)kNoRow ? r1 : 0];
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int r0 = (int)(rv[s] & 0xFFFF), r1 = (int)(rv[s] >> 16);
        A g0 = A(0), g1 = A(0);
        if (r0 != (int)kNoRow) g0 = cur.a[s][0] * ent(cur.j[s][0], cur.u[s][0] * xr[s][0]);
        if (r1 != (int)kNoRow) g1 = cur.a[s][1] * ent(cur.j[s][1], cur.u[s][1] * xr[s][1]);
        flush_pairs(r0, r1, g0, g1, flush);
    }
}

// Process one batch without divergent branches: every lane issues the same
// LDS operations, and an operation a lane must not make is sent to its own
// dummy sum (s_dummy[lane], a value nobody reads) with a zero addend.  Used
// by tiles that hold their own rows and window in LDS (PRIVATE), where
// index(j) maps every column of the tile's entries to its LDS slot; entries
// outside the tile (kNoRow) never reach index's result.  Divergent `if`s in
// the batch cost exec-mask bookkeeping and branches on every entry; here a
// batch is straight-line code.
template <class VT, bool NT, int NP, class Index>
__device__ __forceinline__ void process_batch_flat(const PairBatch<VT, NT, NP> &cur, int qb,
                                                   const Entries<VT, NT> &E, const uint16_t *__restrict__ s_rid,
                                                   const typename VT::A *s_x, typename VT::S *s_y,
                                                   typename VT::S *s_dummy, Index index)
{
    using A = typename VT::A;
    using S = typename VT::S;
    const int half = 2 * (int)blockDim.x;
    const int kb = E.kb, k1 = E.ke;
    const int lane = (int)(threadIdx.x & 63);
    S *const dmy = s_dummy + lane;
    // the row-id table holds ids [0, (k1 - kb + 3) & ~1): a lane past k1
    // reads the last pair (the first, for an empty range), then takes kNoRow
    // (values computed first and selected, so the compiler emits no branch)
    const int plast = max(0, ((k1 - kb + 1) & ~1) - 2);
    const bool quad_lead = (lane & 3) == 0;
#pragma unroll
    for (int s = 0; s < NP; ++s) {
        const int q = qb + half * s;
        const uint32_t w = *reinterpret_cast<const uint32_t *>(s_rid + min(q - kb, plast));
        const uint32_t rv = q < k1 ? w : 0xFFFFFFFFu;
        const int r0 = (int)(rv & 0xFFFF), r1 = (int)(rv >> 16);
        const bool v0 = r0 != (int)kNoRow, v1 = r1 != (int)kNoRow;
        // x of the entries' own rows and of their columns (LDS slots); an
        // entry that is not the tile's reads slot 0 and adds to the dummy,
        // whatever its value
        const int i0 = index(cur.j[s][0]), i1 = index(cur.j[s][1]);
        const int ix0 = v0 ? i0 : 0, ix1 = v1 ? i1 : 0;
        const A xr0 = s_x[v0 ? r0 : 0], xr1 = s_x[v1 ? r1 : 0];
        const A xc0 = s_x[ix0], xc1 = s_x[ix1];
        // scatter au x_r into sum j
        atomic_add(v0 ? &s_y[ix0] : dmy, (S)(cur.au(s, 0) * xr0));
        atomic_add(v1 ? &s_y[ix1] : dmy, (S)(cur.au(s, 1) * xr1));
        // row sums: the pair's two products go to their rows; when the four
        // lanes of an aligned quad each hold a pair of one and the same row
        // (rows do not decrease along the lanes, so the quad's first and
        // last lane decide), the quad's first lane adds the quad's total
        const A g0 = cur.al(s, 0) * xc0, g1 = cur.al(s, 1) * xc1;
        const bool one = (r0 == r1) & v0;
        const int key = one ? r0 : -1 - lane;
        const bool quad = dpp<kDppQuadFirst>(key) == dpp<kDppQuadLast>(key);
        const A v = g0 + g1;
        A vq = v + dpp<kDppXor1>(v);
        vq = vq + dpp<kDppXor2>(vq);
        const bool ta = (quad ? quad_lead : true) & v0;
        const A va = quad ? vq : (one ? v : g0);
        atomic_add(ta ? &s_y[r0] : dmy, (S)va);
        const bool tb = !one & v1;
        atomic_add(tb ? &s_y[r1] : dmy, (S)g1);
    }
}

// Stream entries [kb, k1) of E (kb = k0 rounded down to even).  `cur` holds
// the first batch, issued by the caller before its staging; each batch is
// processed (proc(batch, q)) while the next one loads.  The two batches
// alternate roles (the loop is unrolled by two), so no batch is copied
// between registers.  The batch loop runs the same number of times in every
// lane (lanes past k1 see only kNoRow), so after_first() is called once, by
// all lanes together, after the first batch.
template <class Bt, class Ent, class Proc, class Hook = NoHook>
__device__ __forceinline__ void stream_batches(Bt &cur, const Ent &E, Proc proc, Hook after_first = Hook())
{
    const int step = Bt::kPairs * 2 * (int)blockDim.x;
    const int kb = E.kb, k1 = E.ke;
    Bt nxt;
    int base = kb;
    for (;;) {
        const int qa = base + 2 * (int)threadIdx.x;
        if (base + step < k1) nxt.load(qa + step, E);
        proc(cur, qa);
        if (base == kb) after_first();
        base += step;
        if (base >= k1) break;
        const int qc = base + 2 * (int)threadIdx.x;
        if (base + step < k1) cur.load(qc + step, E);
        proc(nxt, qc);
        base += step;
        if (base >= k1) break;
    }
}

template <class VT, bool LOAD_AU, bool NT, int NP, class NeedAu, class Ent, class Flush, class Hook = NoHook>
__device__ __forceinline__ void own_stream(Batch<VT, true, LOAD_AU, NT, NP> &cur, const Entries<VT, NT> &E,
                                           const uint16_t *__restrict__ s_rid, const typename VT::A *s_x,
                                           NeedAu need_au, Ent ent, Flush flush, Hook after_first = Hook())
{
    stream_batches(
        cur, E,
        [&](Batch<VT, true, LOAD_AU, NT, NP> &b, int q) {
            process_batch<VT, LOAD_AU, NT>(b, q, E, s_rid, s_x, need_au, ent, flush);
        },
        after_first);
}

// Stage a tile's own rows: s_x[i] = x_i and s_y[i] = ad_i x_i (the diagonal
// term starts every row sum).
template <class VT>
__device__ __forceinline__ void stage_rows(int r0, int T, const typename VT::V *__restrict__ ad,
                                           const typename VT::X *__restrict__ x, typename VT::A *s_x,
                                           typename VT::S *s_y, int64_t ldx = 1)
{
    using A = typename VT::A;
    for (int i = threadIdx.x; i < T; i += blockDim.x) {
        const A xv = (A)x[(r0 + i) * ldx];
        s_x[i] = xv;
        s_y[i] = (A)ldv(ad, r0 + i) * xv;
    }
}

// ----------------------------------------------------------------- ATOMIC

// Atomic scatter (Sec. 3 lists atomic primitives as the direct fix of the
// race): y cleared first; scatters into the tile's own rows and the row sums
// meet in LDS, every scatter below the tile is a global atomic add, and each
// own row is added to y with one global atomic at the end.
template <class VT, class YT>
__global__ __launch_bounds__(512) void k_atomic(const int32_t *__restrict__ tiles,
                                                const int32_t *__restrict__ tile_k, int64_t kend,
                                                const int32_t *__restrict__ ia,
                                                const int32_t *__restrict__ ja,
                                                const typename VT::V *__restrict__ ad,
                                                const typename VT::V *__restrict__ al,
                                                const typename VT::V *__restrict__ au,
                                                const typename VT::X *__restrict__ x, int64_t ldx,
                                                YT *__restrict__ y, int64_t ldy, int tmax)
{
    using A = typename VT::A;
    using S = typename VT::S;
    extern __shared__ __align__(16) unsigned char lds[];
    A *s_x = reinterpret_cast<A *>(lds);
    S *s_y = reinterpret_cast<S *>(lds + align16((int64_t)tmax * sizeof(A)));
    uint16_t *s_rid = reinterpret_cast<uint16_t *>(lds + lds_xs(tmax, sizeof(A)));
    const int tid = threadIdx.x, B = blockDim.x;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r0 = tiles[t], r1 = tiles[t + 1], T = r1 - r0;
    const int k0 = tile_k[t], k1 = tile_k[t + 1], kb = k0 & ~1;
    const Entries<VT, true> E(ja, al, au, kb, k1);
    Batch<VT, true, true, true> first;
    first.load(kb + 2 * tid, E);
    stage_rows<VT>(r0, T, ad, x, s_x, s_y, ldx);
    fill_row_ids(ia, r0, r1, kb, s_rid);
    __syncthreads();
    settle_loads();
    own_stream<VT, true, true>(
        first, E, s_rid, s_x, [](int) { return true; },
        [&](int j, A w) -> A {
            if (j >= r0) {
                atomic_add(&s_y[j - r0], w);
                return s_x[j - r0];
            }
            atomic_add(&y[j * ldy], (YT)w);
            return (A)x[j * ldx];
        },
        [&](int r, A v) { atomic_add(&s_y[r], v); });
    __syncthreads();
    for (int i = tid; i < T; i += B) atomic_add(&y[(r0 + i) * ldy], (YT)s_y[i]);
}

// ---------------------------------------------------------------- PRIVATE

// What a tile needs before it can stream, held in registers until it is
// written to LDS: its bounds, its own rows (x, diagonal, row starts; row
// i = threadIdx.x + s * blockDim.x, s < S), its interval list (interval l in
// lane l of every wave: at most 64 intervals) and its window x values (slot
// threadIdx.x + s * blockDim.x, s < S).  Every load whose address is known is
// issued at once, so a tile costs one dependent round trip (intervals, then
// window x) instead of one per staging step.
constexpr int kRegIntervals = kRecIntervals;
typedef int i8v __attribute__((ext_vector_type(8)));
static_assert(kRegIntervals == 8, "i8v holds the record intervals");

template <class VT, int S>
struct NextTile {
    using A = typename VT::A;
    int r0, T, k0, k1, kb, e0, NI, W;
    bool tail;
    int64_t goff;
    i8v rrow, rslot;          // the record's first intervals (uniform)
    A xr[S], dr[S];
    int q0[S], q1[S];
    int ivrow, ivslot;        // lane l: interval l, when there are more than kRegIntervals
    A xw[S];

    // Read the tile record (scalar loads) and issue every load whose
    // address it gives.  Tiles with more than kRegIntervals intervals also
    // load the interval list, one interval per lane.
    __device__ __forceinline__ void issue(const PlanDev &P, int t, const int32_t *__restrict__ ia,
                                          const typename VT::V *__restrict__ ad,
                                          const typename VT::X *__restrict__ x)
    {
        const int tid = threadIdx.x, lane = tid & 63, B = blockDim.x;
        const TileRec *R = P.trec + t;
        r0 = R->r0;
        T = R->r1 - r0;
        k0 = R->k0;
        k1 = R->k1;
        kb = k0 & ~1;
        e0 = R->e0;
        NI = R->ni;
        W = R->w;
        tail = R->tail != 0;
        goff = R->goff;
        rrow = *reinterpret_cast<const i8v *>(R->ivrow);
        rslot = *reinterpret_cast<const i8v *>(R->ivslot);
        ivrow = 0;
        ivslot = 0x7FFFFFFF;
        if (NI > kRegIntervals && lane < NI) {
            ivrow = P.iv_row[e0 + lane];
            ivslot = P.iv_slot[e0 + lane];
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tid + s * B;
            if (i < T) {
                xr[s] = (A)x[r0 + i];
                dr[s] = (A)ldv(ad, r0 + i);
                q0[s] = ia[r0 + i];
                q1[s] = ia[r0 + i + 1];
            }
        }
    }

    // Row of window slot sl: the slot lies in the last interval whose first
    // slot is <= sl, found by compares over the record's intervals, or by a
    // binary search over the lanes (every lane of the wave takes part).
    __device__ __forceinline__ int window_row(int sl) const
    {
        if (NI <= kRegIntervals) {
            int a = rrow[0], b = rslot[0];
#pragma unroll
            for (int k = 1; k < kRegIntervals; ++k) {
                const bool in = sl >= rslot[k];
                a = in ? rrow[k] : a;
                b = in ? rslot[k] : b;
            }
            return a + (sl - b);
        }
        int k = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1) {
            const int c = k + step;
            const int sc = __shfl(ivslot, c & 63);
            if (c < NI && sc <= sl) k = c;
        }
        return __shfl(ivrow, k) + (sl - __shfl(ivslot, k));
    }

    // Window x loads of the first S blockDim.x slots (needs the intervals).
    __device__ __forceinline__ void window(const typename VT::X *__restrict__ x)
    {
        const int tid = threadIdx.x, B = blockDim.x;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int sl = tid + s * B;
            const int row = window_row(sl);
            if (sl < W) xw[s] = (A)x[row];
        }
    }

    // Write the tile into LDS (layout of k_private).  Rows and slots past
    // the first S blockDim.x are loaded here.  Every thread calls it.
    __device__ __forceinline__ void stage(const int32_t *__restrict__ ia, const typename VT::V *__restrict__ ad,
                                          const typename VT::X *__restrict__ x, A *s_x, typename VT::S *s_y,
                                          A *s_xw, typename VT::S *s_w, uint16_t *s_rid,
                                          int32_t *s_ivrow) const
    {
        const int tid = threadIdx.x, B = blockDim.x;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int i = tid + s * B;
            if (i < T) {
                s_x[i] = xr[s];
                s_y[i] = dr[s] * xr[s];
                for (int q = q0[s]; q < q1[s]; ++q) s_rid[q - kb] = (uint16_t)i;
            }
        }
        for (int i = tid + S * B; i < T; i += B) {
            const A xv = (A)x[r0 + i];
            s_x[i] = xv;
            s_y[i] = (A)ldv(ad, r0 + i) * xv;
            const int b = ia[r0 + i], e = ia[r0 + i + 1];
            for (int q = b; q < e; ++q) s_rid[q - kb] = (uint16_t)i;
        }
        const int len = ((k1 - kb) + 3) & ~1;
        for (int q = tid; q < k0 - kb; q += B) s_rid[q] = kNoRow;
        for (int q = (k1 - kb) + tid; q < len; q += B) s_rid[q] = kNoRow;
        if (NI > kRegIntervals && tid < NI) {
            s_ivrow[tid] = ivrow;
            s_ivrow[NI + tid] = ivslot;
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const int sl = tid + s * B;
            if (sl < W) {
                s_xw[sl] = xw[s];
                s_w[sl] = 0;
            }
        }
        for (int base = S * B; base < W; base += B) {
            const int sl = base + tid;
            const int row = window_row(sl);
            if (sl < W) {
                s_xw[sl] = (A)x[row];
                s_w[sl] = 0;
            }
        }
    }
};


// Window slot of a column j below the tile (j in one of the tile's
// intervals).  With at most kRegIntervals intervals, their first rows and
// slot offsets sit in scalar registers (read from the lanes of a NextTile
// that hold them) and the slot is found by compares, without LDS traffic;
// otherwise by a binary search over the LDS copy of the interval list.
// NC > 1 is the most intervals the caller has checked the tile to have (at
// most kRegIntervals): the compares stop there.
template <int NC = kRegIntervals>
struct WindowMap {
    static_assert(NC > 1 && NC <= kRegIntervals, "compares over the record's intervals");
    int n;
    i8v row, off;   // vector types keep the table in registers
    const int32_t *s_ivrow, *s_ivslot;

    template <class NT>
    __device__ __forceinline__ void init(const NT &nt, const int32_t *s_iv)
    {
        n = nt.NI;
        s_ivrow = s_iv;
        s_ivslot = s_iv + nt.NI;
        row = nt.rrow;
        off = nt.rslot - nt.rrow;   // unused entries: INT32_MAX rows, never selected
    }

    __device__ __forceinline__ int slot(int j) const
    {
        if (NC < kRegIntervals || n <= kRegIntervals) {
            int o = off[0];
#pragma unroll
            for (int k = 1; k < NC; ++k) o = j >= row[k] ? off[k] : o;
            return j + o;
        }
        const int k = upper_index(s_ivrow, n, j);
        return s_ivslot[k] + (j - s_ivrow[k]);
    }

    // LDS index of column j in a tile of T rows from r0 whose window slots
    // follow its rows: j - r0 for an own row, T + slot(j) below.  The own
    // range is one more interval start of the compare chain.
    __device__ __forceinline__ int local(int j, int r0, int T) const
    {
        if (NC < kRegIntervals || n <= kRegIntervals) {
            int o = off[0] + T;
#pragma unroll
            for (int k = 1; k < NC; ++k) o = j >= row[k] ? off[k] + T : o;
            o = j >= r0 ? -r0 : o;
            return j + o;
        }
        return j >= r0 ? j - r0 : T + slot(j);
    }
};

// Local buffers of Sec. 3.1 kept in LDS: a tile of rows [r0, r1) accumulates
// its own rows (s_y) and its effective range below r0 (s_w, compact window
// slots).  x of both ranges is staged in LDS first (s_x, s_xw).  Own rows go
// to y; window slots go to the partial buffer for the merge pass.  All
// staging loads and the first batch of entries are in flight together.
// Ways a tile's sums reach y (MODE):
//   kMergePass   own rows stored, window slots to the partial buffer;
//   kMergeAtomic y is zero beforehand and both the own rows and the window
//                slots are added to y with global atomics; no partials;
//   kMergeColor  y is zero beforehand; the launch runs one colour class of
//                tiles (tlist), whose written rows are disjoint, so both are
//                added to y with plain read-modify-writes.
// Pairs per lane in one batch of the PRIVATE stream.  Three or four pairs
// put more bytes in flight per wave but cost registers (89 and 115 VGPRs for
// FP64 against 63) and measured slower on the 27-point and tetrahedral
// meshes, so two.
constexpr int kPrivatePairs = 2;

constexpr int kMergePass = 0, kMergeAtomic = 1, kMergeColor = 2;


// NC: the plan's largest number of window intervals of one tile is at most
// NC (2, 4 or kRegIntervals): the window lookup makes NC - 1 compares.
template <class VT, class YT, int MODE, int NC>
__device__ __forceinline__ void private_tile(PlanDev P, const int32_t *__restrict__ tlist,
                                                 const int32_t *__restrict__ ia,
                                                 const int32_t *__restrict__ ja,
                                                 const typename VT::V *__restrict__ ad,
                                                 const typename VT::V *__restrict__ al,
                                                 const typename VT::V *__restrict__ au,
                                                 const typename VT::X *__restrict__ x,
                                                 YT *__restrict__ y, int smax, int emax)
{
    using A = typename VT::A;
    using S = typename VT::S;
    extern __shared__ __align__(16) unsigned char lds[];
    // x of the T own rows then the window slots; sums likewise: an entry's
    // target is one index into both
    A *s_x = reinterpret_cast<A *>(lds);
    S *s_y = reinterpret_cast<S *>(lds + align16((int64_t)smax * sizeof(A)));
    uint16_t *s_rid = reinterpret_cast<uint16_t *>(lds + lds_xs(smax, sizeof(A)));
    // one dummy sum per lane (process_batch_flat), then the interval list
    S *s_dummy = reinterpret_cast<S *>(reinterpret_cast<unsigned char *>(s_rid) + align16(((int64_t)emax + 4) * 2));
    int32_t *s_ivrow = reinterpret_cast<int32_t *>(s_dummy + kDummySums);

    const int tid = threadIdx.x, B = blockDim.x;
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int t = MODE == kMergeColor ? tlist[b] : b;
    NextTile<VT, 2> nt;
    nt.issue(P, t, ia, ad, x);
    A *s_xw = s_x + nt.T;
    S *s_w = s_y + nt.T;
    // The value ranges are read as padded pairs (Entries).  The one tile
    // whose range ends in a bfloat16 pair past the last stored entry of the
    // matrix (tail) streams all but that entry and adds its two products
    // itself after the stream.
    const Entries<VT, true> E(ja, al, au, nt.kb, nt.tail ? nt.k1 - 1 : nt.k1, true);
    const bool tail = nt.tail && nt.k1 - 1 >= nt.k0;
    PairBatch<VT, true, kPrivatePairs> first;
    first.load(nt.kb + 2 * tid, E);
    nt.window(x);
    nt.stage(ia, ad, x, s_x, s_y, s_xw, s_w, s_rid, s_ivrow);
    const int r0 = nt.r0, T = nt.T, W = nt.W;
    __syncthreads();
    settle_loads();

    WindowMap<NC> wm;
    wm.init(nt, s_ivrow);
    auto index = [&, wm](int j) -> int { return wm.local(j, r0, T); };
    stream_batches(first, E, [&](PairBatch<VT, true, kPrivatePairs> &bt, int q) {
        process_batch_flat<VT, true>(bt, q, E, s_rid, s_x, s_y, s_dummy, index);
    });
    if (tail && tid == 0) {
        const int q = nt.k1 - 1;
        const int rr = s_rid[q - nt.kb], idx = index(ja[q]);
        atomic_add(&s_y[idx], (S)((A)ldv(au, q) * s_x[rr]));
        atomic_add(&s_y[rr], (S)((A)ldv(al, q) * s_x[idx]));
    }
    __syncthreads();

    if (MODE == kMergeAtomic) {
        for (int i = tid; i < T; i += B) atomic_add(&y[r0 + i], (YT)s_y[i]);
        for (int base = 0; base < W; base += B) {
            const int sl = base + tid;
            const int row = nt.window_row(sl);   // every lane takes part
            if (sl < W) atomic_add(&y[row], (YT)s_w[sl]);
        }
        return;
    }
    if (MODE == kMergeColor) {
        for (int i = tid; i < T; i += B) y[r0 + i] += (YT)s_y[i];
        for (int base = 0; base < W; base += B) {
            const int sl = base + tid;
            const int row = nt.window_row(sl);   // every lane takes part
            if (sl < W) y[row] += (YT)s_w[sl];
        }
        return;
    }
    for (int i = tid; i < T; i += B) y[r0 + i] = (YT)s_y[i];
    if (W) {
        A *part = reinterpret_cast<A *>(P.partials) + nt.goff;
        for (int sl = tid; sl < W; sl += B) part[sl] = (A)s_w[sl];
    }
}

template <class VT, class YT, int MODE, int NC = kRegIntervals>
__global__ __launch_bounds__(512) void k_private(PlanDev P, const int32_t *__restrict__ tlist,
                                                 const int32_t *__restrict__ ia,
                                                 const int32_t *__restrict__ ja,
                                                 const typename VT::V *__restrict__ ad,
                                                 const typename VT::V *__restrict__ al,
                                                 const typename VT::V *__restrict__ au,
                                                 const typename VT::X *__restrict__ x,
                                                 YT *__restrict__ y, int smax, int emax)
{
    private_tile<VT, YT, MODE, NC>(P, tlist, ia, ja, ad, al, au, x, y, smax, emax);
}

// ------------------------------------------------- PRIVATE, both products

// y = A x and yt = A^T x in one pass over the entries.  The transpose
// product is the same loop with al and au exchanged (Sec. 5), so per entry
// (i, j): y_i += al x_j, y_j += au x_i, yt_i += au x_j and yt_j += al x_i.
// One batch: ent2(j, wy, wt) scatters wy into the sums of y and wt into
// those of yt at column j and returns x_j; the gathered products go to
// flush_y and flush_t.
template <class VT, class Ent2, class FlushY, class FlushT>
__device__ __forceinline__ void process_batch_pair(Batch<VT, true, true, true> &cur, int qb,
                                                   const Entries<VT, true> &E, const uint16_t *__restrict__ s_rid,
                                                   const typename VT::A *s_x, Ent2 ent2, FlushY flush_y,
                                                   FlushT flush_t)
{
    using A = typename VT::A;
    const int half = 2 * (int)blockDim.x;
    const int kb = E.kb, k1 = E.ke;
    uint32_t rv[2];
    A xr[2][2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int q = qb + half * s;
        rv[s] = q < k1 ? *reinterpret_cast<const uint32_t *>(s_rid + (q - kb)) : 0xFFFFFFFFu;
        const int r0 = (int)(rv[s] & 0xFFFF), r1 = (int)(rv[s] >> 16);
        xr[s][0] = s_x[r0 != (int)kNoRow ? r0 : 0];
        xr[s][1] = s_x[r1 != (int)kNoRow ? r1 : 0];
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int r0 = (int)(rv[s] & 0xFFFF), r1 = (int)(rv[s] >> 16);
        A gy0 = A(0), gy1 = A(0), gt0 = A(0), gt1 = A(0);
        if (r0 != (int)kNoRow) {
            const A xj = ent2(cur.j[s][0], cur.u[s][0] * xr[s][0], cur.a[s][0] * xr[s][0]);
            gy0 = cur.a[s][0] * xj;
            gt0 = cur.u[s][0] * xj;
        }
        if (r1 != (int)kNoRow) {
            const A xj = ent2(cur.j[s][1], cur.u[s][1] * xr[s][1], cur.a[s][1] * xr[s][1]);
            gy1 = cur.a[s][1] * xj;
            gt1 = cur.u[s][1] * xj;
        }
        flush_pairs(r0, r1, gy0, gy1, flush_y);
        flush_pairs(r0, r1, gt0, gt1, flush_t);
    }
}

// PRIVATE tile producing both products (atomic merge: y and yt are cleared
// beforehand; every tile adds its own rows and window sums to both with
// global atomics).  LDS: x of own rows then window slots, the sums of y and
// of yt likewise, row ids, interval list.
template <class VT, class YT>
__global__ __launch_bounds__(512) void k_private_pair(PlanDev P, const int32_t *__restrict__ ia,
                                                      const int32_t *__restrict__ ja,
                                                      const typename VT::V *__restrict__ ad,
                                                      const typename VT::V *__restrict__ al,
                                                      const typename VT::V *__restrict__ au,
                                                      const typename VT::X *__restrict__ x, YT *__restrict__ y,
                                                      YT *__restrict__ yt, int smax, int emax)
{
    using A = typename VT::A;
    using S = typename VT::S;
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t sbytes = align16((int64_t)smax * sizeof(S));
    A *s_x = reinterpret_cast<A *>(lds);
    S *s_y = reinterpret_cast<S *>(lds + align16((int64_t)smax * sizeof(A)));
    S *s_t = reinterpret_cast<S *>(lds + align16((int64_t)smax * sizeof(A)) + sbytes);
    uint16_t *s_rid = reinterpret_cast<uint16_t *>(lds + lds_xs(smax, sizeof(A)) + sbytes);
    int32_t *s_ivrow = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(s_rid) +
                                                   align16(((int64_t)emax + 4) * 2));
    const int tid = threadIdx.x, B = blockDim.x, half = 2 * B;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    NextTile<VT, 2> nt;
    nt.issue(P, t, ia, ad, x);
    A *s_xw = s_x + nt.T;
    S *s_w = s_y + nt.T;
    const Entries<VT, true> E(ja, al, au, nt.kb, nt.k1);
    Batch<VT, true, true, true> cur;
    cur.load(nt.kb + 2 * tid, E);
    nt.window(x);
    nt.stage(ia, ad, x, s_x, s_y, s_xw, s_w, s_rid, s_ivrow);
    const int r0 = nt.r0, T = nt.T, W = nt.W, k1 = nt.k1;
    WindowMap<> wm;
    wm.init(nt, s_ivrow);
    __syncthreads();
    // the transpose has the same diagonal: its sums start as those of y
    for (int i = tid; i < T + W; i += B) s_t[i] = s_y[i];
    __syncthreads();
    settle_loads();

    auto ent2 = [&, wm](int j, A wy, A wt) -> A {
        const int idx = j >= r0 ? j - r0 : T + wm.slot(j);
        atomic_add(&s_y[idx], wy);
        atomic_add(&s_t[idx], wt);
        return s_x[idx];
    };
    auto flush_y = [&](int r, A v) { atomic_add(&s_y[r], v); };
    auto flush_t = [&](int r, A v) { atomic_add(&s_t[r], v); };
    int base = nt.kb;
    do {
        const int qb = base + 2 * tid;
        Batch<VT, true, true, true> nxt;
        if (base + 2 * half < k1) nxt.load(qb + 2 * half, E);
        process_batch_pair<VT>(cur, qb, E, s_rid, s_x, ent2, flush_y, flush_t);
        cur = nxt;
        base += 2 * half;
    } while (base < k1);
    __syncthreads();

    for (int i = tid; i < T; i += B) {
        atomic_add(&y[r0 + i], (YT)s_y[i]);
        atomic_add(&yt[r0 + i], (YT)s_t[i]);
    }
    for (int b0 = 0; b0 < W; b0 += B) {
        const int sl = b0 + tid;
        const int row = nt.window_row(sl);   // every lane takes part
        if (sl < W) {
            atomic_add(&y[row], (YT)s_w[sl]);
            atomic_add(&yt[row], (YT)s_t[T + sl]);
        }
    }
}

// Merge pass: y_i += the partial slots covering row i, in ascending tile
// order.  Merge block b (one workgroup, one row per thread) lists segments
// [lo, hi) with partial index base + i; segments are taken four at a time so
// their partial loads are in flight together.  MT is the merge type; COMP
// adds a TwoSum (Knuth) error term.
template <class A, class YT, class MT, bool COMP>
__global__ __launch_bounds__(kMergeBlock) void k_merge(int32_t n, PlanDev P, YT *__restrict__ y)
{
    constexpr int K = 4;
    const int b = blockIdx.x;
    const int e0 = P.mb_ptr[b], e1 = P.mb_ptr[b + 1];
    const int i = b * kMergeBlock + threadIdx.x;
    if (e0 == e1 || i >= n) return;
    const A *part = reinterpret_cast<const A *>(P.partials);
    MT s = (MT)y[i], c = MT(0);
    for (int e = e0; e < e1; e += K) {
        A v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            v[k] = A(0);
            if (e + k < e1) {
                const MergeSeg g = P.mb_seg[e + k];
                if (i >= g.lo && i < g.hi) v[k] = part[g.base + i];
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (e + k >= e1) break;
            const MT w = (MT)v[k];
            if (COMP) {
                const MT s2 = s + w;
                const MT bp = s2 - s;
                c += (s - (s2 - bp)) + (w - bp);
                s = s2;
            } else {
                s += w;
            }
        }
    }
    y[i] = (YT)(s + c);
}

// ------------------------------------------------------------------ OWNER

// Owner computes: the tile streams its own rows, gathering x from LDS or L2
// and scattering only into its own rows; then it visits, chunk by chunk, the
// rows of later tiles that scatter into it (pull chunks, re-read from cache:
// temporal loads) and adds the entries whose target lies in [r0, r1).  Each y
// entry is completed in one workgroup's LDS and stored once: no partials, no
// atomics outside LDS, no second pass.
template <class VT, class YT>
__global__ __launch_bounds__(512) void k_owner(PlanDev P, int64_t kend, const int32_t *__restrict__ ia,
                                               const int32_t *__restrict__ ja,
                                               const typename VT::V *__restrict__ ad,
                                               const typename VT::V *__restrict__ al,
                                               const typename VT::V *__restrict__ au,
                                               const typename VT::X *__restrict__ x,
                                               YT *__restrict__ y, int tmax, int pmax, int emax)
{
    using A = typename VT::A;
    using S = typename VT::S;
    extern __shared__ __align__(16) unsigned char lds[];
    A *s_x = reinterpret_cast<A *>(lds);
    A *s_xp = s_x + tmax;
    const int64_t xbytes = align16(((int64_t)tmax + pmax) * sizeof(A));
    S *s_y = reinterpret_cast<S *>(lds + xbytes);
    uint16_t *s_rid = reinterpret_cast<uint16_t *>(lds + xbytes + align16((int64_t)tmax * sizeof(S)));

    const int tid = threadIdx.x, B = blockDim.x;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int r0 = P.tiles[t], r1 = P.tiles[t + 1], T = r1 - r0;
    const int k0 = P.tile_k[t], k1 = P.tile_k[t + 1], kb = k0 & ~1;
    const Entries<VT, false> E(ja, al, au, kb, k1);
    Batch<VT, true, false, false> first;
    first.load(kb + 2 * tid, E);
    stage_rows<VT>(r0, T, ad, x, s_x, s_y);
    fill_row_ids(ia, r0, r1, kb, s_rid);
    __syncthreads();
    settle_loads();
    own_stream<VT, false, false>(
        first, E, s_rid, s_x, [&](int j) { return j >= r0; },
        [&](int j, A w) -> A {
            if (j >= r0) {
                atomic_add(&s_y[j - r0], w);
                return s_x[j - r0];
            }
            return (A)x[j];
        },
        [&](int r, A v) { atomic_add(&s_y[r], v); });

    const int p0 = P.iv_ptr[t], p1 = P.iv_ptr[t + 1];
    const int half = 2 * B;
    for (int e = p0; e < p1; ++e) {
        const int pa = P.iv_row[e], L = P.iv_len[e];
        const int qa = ia[pa], qe = ia[pa + L], qbase = qa & ~1;
        const Entries<VT, false> Ep(ja, al, au, qbase, qe);
        Batch<VT, false, false, false> cur;
        cur.load(qbase + 2 * tid, Ep);
        __syncthreads();   // earlier readers of s_rid / s_xp are done
        for (int i = tid; i < L; i += B) s_xp[i] = (A)x[pa + i];
        fill_row_ids(ia, pa, pa + L, qbase, s_rid);
        __syncthreads();
        settle_loads();
        for (int qb = qbase + 2 * tid; qb < qe; qb += 2 * half) {
            Batch<VT, false, false, false> nxt;
            if (qb + 2 * half < qe) nxt.load(qb + 2 * half, Ep);
#pragma unroll
            for (int s = 0; s < 2; ++s) {
                const int q = qb + half * s;
                if (q >= qe) continue;
                const uint32_t rv = *reinterpret_cast<const uint32_t *>(s_rid + (q - qbase));
                const int ra = (int)(rv & 0xFFFF), rb = (int)(rv >> 16);
                const int j0 = cur.j[s][0], j1 = cur.j[s][1];
                const bool t0 = ra != (int)kNoRow && j0 >= r0 && j0 < r1;
                const bool t1 = rb != (int)kNoRow && j1 >= r0 && j1 < r1;
                if (!(t0 || t1)) continue;
                A uv[2];
                Ep.au2(q, uv);
                if (t0) atomic_add(&s_y[j0 - r0], uv[0] * s_xp[ra]);
                if (t1) atomic_add(&s_y[j1 - r0], uv[1] * s_xp[rb]);
            }
            cur = nxt;
        }
    }
    __syncthreads();
    for (int i = tid; i < T; i += B) y[r0 + i] = (YT)s_y[i];
}

// ----------------------------------------------------- multiple right-hand sides
//
// Y = A X for row-major n x r blocks.  Each tile keeps C columns of its rows
// (and of its window slots) in LDS at a time and streams its entries once per
// chunk of C columns; every stored entry is applied to all C columns.  Chunks
// after the first re-read the tile's entries from L2 (temporal loads).

template <class VT> struct MmCols { static constexpr int C = 4; };
template <> struct MmCols<F32T> { static constexpr int C = 8; };
template <> struct MmCols<B16T> { static constexpr int C = 8; };

// Window of a PRIVATE tile read from its record: slot of a column below the
// tile and row of a slot.  With at most kRecIntervals intervals both come
// from compares over the record's interval table (held in registers);
// otherwise from binary searches over the LDS copy of the interval list.
struct RecWindow {
    int n;
    i8v row, slot;                      // unused entries: INT32_MAX
    const int32_t *s_row, *s_slot;

    __device__ __forceinline__ void init(const TileRec *R, const int32_t *s_iv)
    {
        n = R->ni;
        row = *reinterpret_cast<const i8v *>(R->ivrow);
        slot = *reinterpret_cast<const i8v *>(R->ivslot);
        s_row = s_iv;
        s_slot = s_iv + n;
    }
    __device__ __forceinline__ int slot_of(int j) const
    {
        if (n <= kRecIntervals) {
            int o = slot[0] - row[0];
#pragma unroll
            for (int k = 1; k < kRecIntervals; ++k) o = j >= row[k] ? slot[k] - row[k] : o;
            return j + o;
        }
        const int k = upper_index(s_row, n, j);
        return s_slot[k] + (j - s_row[k]);
    }
    __device__ __forceinline__ int row_of(int sl) const
    {
        if (n <= kRecIntervals) {
            int o = row[0] - slot[0];
#pragma unroll
            for (int k = 1; k < kRecIntervals; ++k) o = sl >= slot[k] ? row[k] - slot[k] : o;
            return sl + o;
        }
        const int k = upper_index(s_slot, n, sl);
        return s_row[k] + (sl - s_slot[k]);
    }
};

// One batch of the multi-column stream (lane pairs at qb and qb + 2B): each
// entry of row i (relative) with column j scatters au x_i into the sums at
// index idx = j - r0 (own row) or T + slot(j) (window slot), C columns at
// once, and gathers al x_j; a lane's pair of one row is added to the row's
// sums once.  LDS arrays are column-major with leading dimension ld, so the
// lanes of one instruction touch one column (8-byte stride between indices,
// as in the single-vector kernels) instead of C-wide rows that alias onto a
// few banks.  Columns from nc on are padding and skipped (nc is uniform).
template <class VT, int C, class Batch_>
__device__ __forceinline__ void process_batch_mm(const Batch_ &cur, int qb, int kb, int k1,
                                                 const uint16_t *__restrict__ s_rid, const typename VT::A *s_x,
                                                 typename VT::S *s_y, int ld, int r0, int T, const RecWindow &wm,
                                                 int nc)
{
    using A = typename VT::A;
    using S = typename VT::S;
    const int half = 2 * (int)blockDim.x;
#pragma unroll
    for (int sp = 0; sp < 2; ++sp) {
        const int q = qb + half * sp;
        const uint32_t rv = q < k1 ? *reinterpret_cast<const uint32_t *>(s_rid + (q - kb)) : 0xFFFFFFFFu;
        const int ra = (int)(rv & 0xFFFF), rb = (int)(rv >> 16);
        A g[2][C];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int row = h ? rb : ra;
#pragma unroll
            for (int c = 0; c < C; ++c) g[h][c] = A(0);
            if (row == (int)kNoRow) continue;
            const int j = cur.j[sp][h];
            const int idx = j >= r0 ? j - r0 : T + wm.slot_of(j);
            A xi[C], xj[C];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                xi[c] = s_x[c * ld + row];
                xj[c] = s_x[c * ld + idx];
            }
            const A a = cur.a[sp][h], u = cur.u[sp][h];
#pragma unroll
            for (int c = 0; c < C; ++c) {
                if (c < nc) atomic_add(&s_y[c * ld + idx], (S)(u * xi[c]));
                g[h][c] = a * xj[c];
            }
        }
        if (ra == rb) {
            if (ra != (int)kNoRow) {
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (c < nc) atomic_add(&s_y[c * ld + ra], (S)(g[0][c] + g[1][c]));
            }
        } else {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int row = h ? rb : ra;
                if (row == (int)kNoRow) continue;
#pragma unroll
                for (int c = 0; c < C; ++c)
                    if (c < nc) atomic_add(&s_y[c * ld + row], (S)g[h][c]);
            }
        }
    }
}

// One PRIVATE tile t of a product with r columns (r >= 1), C columns at a
// time; chunks after the first re-read the tile's entries from L2 (temporal
// loads).  LDS: x of the T own rows then the W window slots, one column after
// the other (leading dimension mm_ld(smax)); the FP64 sums likewise; row ids;
// the interval list when the tile has more intervals than its record holds.  Own rows go to Y, window sums to the
// partial buffer (r values per slot) for the merge pass.  Used by the
// multi-column kernel and by the batched persistent kernel.
template <class VT, class YT>
__device__ __forceinline__ void private_tile_mm(const PlanDev &P, int t, const int32_t *__restrict__ ia,
                                                const int32_t *__restrict__ ja,
                                                const typename VT::V *__restrict__ ad,
                                                const typename VT::V *__restrict__ al,
                                                const typename VT::V *__restrict__ au,
                                                const typename VT::X *__restrict__ X, int64_t ldx,
                                                YT *__restrict__ Y, int64_t ldy, int r, int smax, int emax,
                                                unsigned char *lds)
{
    using A = typename VT::A;
    using S = typename VT::S;
    constexpr int C = MmCols<VT>::C;
    const int ld = mm_ld(smax);
    const int64_t nv = (int64_t)ld * C;
    A *s_x = reinterpret_cast<A *>(lds);
    S *s_y = reinterpret_cast<S *>(lds + align16(nv * sizeof(A)));
    uint16_t *s_rid = reinterpret_cast<uint16_t *>(lds + lds_xs(nv, sizeof(A)));
    int32_t *s_iv = reinterpret_cast<int32_t *>(reinterpret_cast<unsigned char *>(s_rid) +
                                                align16(((int64_t)emax + 4) * 2));
    const int tid = threadIdx.x, B = blockDim.x, half = 2 * B;
    const TileRec *R = P.trec + t;
    const int r0 = R->r0, T = R->r1 - r0, k0 = R->k0, k1 = R->k1, kb = k0 & ~1;
    const int e0 = R->e0, NI = R->ni, W = R->w;
    const int64_t goff = R->goff;
    __syncthreads();   // the workgroup's previous use of LDS is finished
    if (NI > kRecIntervals) {
        for (int i = tid; i < NI; i += B) {
            s_iv[i] = P.iv_row[e0 + i];
            s_iv[NI + i] = P.iv_slot[e0 + i];
        }
    }
    fill_row_ids(ia, r0, r0 + T, kb, s_rid);
    RecWindow wm;
    wm.init(R, s_iv);
    __syncthreads();   // the interval list is visible to the window staging
    const Entries<VT, false> E(ja, al, au, kb, k1);
    for (int cc = 0; cc < r; cc += C) {
        const int nc = min(C, r - cc);
        if (cc) __syncthreads();   // the previous chunk's readers are done
        Batch<VT, true, true, false> cur;
        cur.load(kb + 2 * tid, E);
        // staging: U elements per thread at a time, their loads in flight
        // together (row i < T: own row r0 + i; else window slot i - T)
        constexpr int U = 8;
        const int ne = (T + W) * C;
        for (int e0 = tid; e0 < ne; e0 += U * B) {
            A xv[U], dv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * B;
                const int i = e / C, c = e % C;
                xv[u] = A(0);
                dv[u] = A(0);
                if (e < ne) {
                    const int row = i < T ? r0 + i : wm.row_of(i - T);
                    if (c < nc) xv[u] = (A)X[(int64_t)row * ldx + cc + c];
                    if (i < T) dv[u] = (A)ldv(ad, row);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * B;
                if (e < ne) {
                    const int i = e / C, c = e % C;
                    s_x[c * ld + i] = xv[u];
                    s_y[c * ld + i] = dv[u] * xv[u];
                }
            }
        }
        __syncthreads();
        settle_loads();
        int base = kb;
        do {
            const int qb = base + 2 * tid;
            Batch<VT, true, true, false> nxt;
            if (base + 2 * half < k1) nxt.load(qb + 2 * half, E);
            process_batch_mm<VT, C>(cur, qb, kb, k1, s_rid, s_x, s_y, ld, r0, T, wm, nc);
            cur = nxt;
            base += 2 * half;
        } while (base < k1);
        __syncthreads();
        for (int e = tid; e < T * C; e += B) {
            const int i = e / C, c = e % C;
            if (c < nc) Y[(int64_t)(r0 + i) * ldy + cc + c] = (YT)s_y[c * ld + i];
        }
        if (W) {
            A *part = reinterpret_cast<A *>(P.partials);
            for (int e = tid; e < W * C; e += B) {
                const int sl = e / C, c = e % C;
                if (c < nc) part[(goff + sl) * r + cc + c] = (A)s_y[c * ld + T + sl];
            }
        }
    }
}

template <class VT, class YT>
__global__ __launch_bounds__(512) void k_private_mm(PlanDev P, const int32_t *__restrict__ ia,
                                                    const int32_t *__restrict__ ja,
                                                    const typename VT::V *__restrict__ ad,
                                                    const typename VT::V *__restrict__ al,
                                                    const typename VT::V *__restrict__ au,
                                                    const typename VT::X *__restrict__ X, int64_t ldx,
                                                    YT *__restrict__ Y, int64_t ldy, int r, int smax, int emax)
{
    extern __shared__ __align__(16) unsigned char lds[];
    private_tile_mm<VT, YT>(P, xcd_tile(blockIdx.x, gridDim.x), ia, ja, ad, al, au, X, ldx, Y, ldy, r, smax, emax,
                            lds);
}

// Merge pass for r columns: Y[i, c] += the partial slots covering row i, in
// ascending tile order (partial slot g holds r values).  One thread per
// (row, column), U of them per thread at a time; segments are taken K at a
// time, so up to U K partial loads are in flight together.
template <class A, class YT, class MT, bool COMP>
__device__ __forceinline__ void merge_block_mm(int32_t n, const PlanDev &P, YT *__restrict__ Y, int64_t ldy,
                                               int r, int b)
{
    constexpr int K = 4, U = 4;
    const int e0 = P.mb_ptr[b], e1 = P.mb_ptr[b + 1];
    if (e0 == e1) return;
    const A *part = reinterpret_cast<const A *>(P.partials);
    const int rows = min(kMergeBlock, n - b * kMergeBlock);
    const int ne = rows * r;
    const int B = blockDim.x;
    for (int f0 = threadIdx.x; f0 < ne; f0 += U * B) {
        int i[U], c[U];
        MT s[U], cm[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int f = min(f0 + u * B, ne - 1);   // clamped lanes repeat a valid element, not stored
            i[u] = b * kMergeBlock + f / r;
            c[u] = f % r;
            s[u] = (MT)Y[(int64_t)i[u] * ldy + c[u]];
            cm[u] = MT(0);
        }
        for (int g0 = e0; g0 < e1; g0 += K) {
            A v[K][U];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const MergeSeg g = P.mb_seg[min(g0 + k, e1 - 1)];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    v[k][u] = A(0);
                    if (g0 + k < e1 && i[u] >= g.lo && i[u] < g.hi) v[k][u] = part[(g.base + i[u]) * r + c[u]];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (g0 + k >= e1) break;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const MT w = (MT)v[k][u];
                    if (COMP) {
                        const MT s2 = s[u] + w;
                        const MT bp = s2 - s[u];
                        cm[u] += (s[u] - (s2 - bp)) + (w - bp);
                        s[u] = s2;
                    } else {
                        s[u] += w;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (f0 + u * B < ne) Y[(int64_t)i[u] * ldy + c[u]] = (YT)(s[u] + cm[u]);
    }
}

template <class A, class YT, class MT, bool COMP>
__global__ __launch_bounds__(kMergeBlock) void k_merge_mm(int32_t n, PlanDev P, YT *__restrict__ Y,
                                                          int64_t ldy, int r)
{
    merge_block_mm<A, YT, MT, COMP>(n, P, Y, ldy, r, blockIdx.x);
}

// ----------------------------------------------------------------- batched
//
// Many independent products in one persistent launch: the work list holds
// (matrix, tile) items sorted by decreasing cost, and each workgroup walks it
// with a grid stride; a second launch merges the window partials of every
// matrix (work list of (matrix, merge block)).  Both launches read only the
// bound workspace, so they can be recorded into a HIP graph.

template <class VT, class YT>
__global__ __launch_bounds__(512) void k_batch_tiles(const MatDev *__restrict__ mats, const int2 *__restrict__ items,
                                                     int nitems, int transpose, int smax, int emax)
{
    extern __shared__ __align__(16) unsigned char lds[];
    using V = typename VT::V;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 w = items[it];
        const MatDev &M = mats[w.x];
        const V *al = static_cast<const V *>(transpose ? M.au : M.al);
        const V *au = static_cast<const V *>(transpose ? M.al : M.au);
        private_tile_mm<VT, YT>(M.P, w.y, M.ia, M.ja, static_cast<const V *>(M.ad), al, au,
                                static_cast<const typename VT::X *>(M.X), M.ldx, static_cast<YT *>(M.Y), M.ldy,
                                M.r, smax, emax, lds);
    }
}

template <class A, class YT, class MT, bool COMP>
__global__ __launch_bounds__(kMergeBlock) void k_batch_merge(const MatDev *__restrict__ mats,
                                                             const int2 *__restrict__ items, int nitems)
{
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 w = items[it];
        const MatDev &M = mats[w.x];
        merge_block_mm<A, YT, MT, COMP>(M.n, M.P, static_cast<YT *>(M.Y), M.ldy, M.r, w.y);
    }
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
                                               const typename VT::X *__restrict__ x, int64_t ldx,
                                               YT *__restrict__ y, int64_t ldy)
{
    using A = typename VT::A;
    const int lg = threadIdx.x % G;
    const int grp = blockIdx.x * (blockDim.x / G) + threadIdx.x / G;
    const int ngrp = gridDim.x * (blockDim.x / G);
    rows_loop<G, typename VT::V, A>(
        c0, c1, grp, ngrp, lg, [&](int idx) { return crow[idx]; }, [&](int r) { return ia[r]; },
        [&](int r) { return (A)x[r * ldx]; }, [&](int r) { return (A)ldv(ad, r); }, ja, al, au,
        [&](int j, A a, A w) -> A {
            y[j * ldy] = y[j * ldy] + (YT)w;
            return a * (A)x[j * ldx];
        },
        [&](int r, A v) { y[r * ldy] = y[r * ldy] + (YT)v; });
}

// --------------------------------------------------------------- dispatch

// Device view of a plan whose tables sit at the workspace ws (partials after them).
static PlanDev plan_dev(const csrc_plan *p, void *ws)
{
    char *b = static_cast<char *>(ws);
    return plan_dev_at(p, b, b ? b + p->t_partials.offset : nullptr);
}

static int device_cus();

// workgroups of k_fill_zero for count values (about 16 per thread; fewer,
// longer workgroups clear a large y fastest)
static int fill_grid(int64_t count) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (count + 4095) / 4096)); }

// The PRIVATE tile kernel for a plan: numerically symmetric storage (au is
// al) loads one value per entry; the window lookup makes as few compares as
// the plan's largest interval count per tile allows.
template <class VT, class YT, int MODE>
static decltype(&k_private<VT, YT, MODE>) private_kernel(const csrc_plan *p, bool sym)
{
    if (p->max_intervals <= 2) return sym ? k_private<SymT<VT>, YT, MODE, 2> : k_private<VT, YT, MODE, 2>;
    if (p->max_intervals <= 4) return sym ? k_private<SymT<VT>, YT, MODE, 4> : k_private<VT, YT, MODE, 4>;
    return sym ? k_private<SymT<VT>, YT, MODE> : k_private<VT, YT, MODE>;
}

template <class VT, class YT, int G>
static int launch_variant(const csrc_plan *p, const csrc_matrix *A, const void *al_, const void *au_,
                          const void *x_, int64_t ldx, void *y_, int64_t ldy, int r, void *ws, hipStream_t s)
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
    const bool single = r == 1 && ldx == 1 && ldy == 1;
    PlanDev P = plan_dev(p, ws);
    auto set_lds = [](const void *kern, size_t lds) {
        return lds > 65536 ? hip_status(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds))
                           : (int)CSRC_OK;
    };
    switch (p->o.variant) {
    case CSRC_V_PLAIN:
        k_fill_zero<YT><<<fill_grid((int64_t)n * r), 256, 0, s>>>(y, n, r, ldy);
        for (int c = 0; c < r; ++c)
            k_plain<VT, YT><<<(n + 255) / 256, 256, 0, s>>>(n, A->ia, A->ja, ad, al, au, x + c, ldx, y + c, ldy);
        break;
    case CSRC_V_ATOMIC: {
        k_fill_zero<YT><<<fill_grid((int64_t)n * r), 256, 0, s>>>(y, n, r, ldy);
        const int tmax = p->max_tile_rows;
        const size_t lds = (size_t)lds_atomic(tmax, p->max_tile_entries, sizeof(Acc));
        auto kern = k_atomic<VT, YT>;
        if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
        for (int c = 0; c < r; ++c)
            kern<<<p->ntiles, B, lds, s>>>(P.tiles, P.tile_k, A->k, A->ia, A->ja, ad, al, au, x + c, ldx, y + c,
                                           ldy, tmax);
        break;
    }
    case CSRC_V_PRIVATE: {
        const int emax = p->max_tile_entries, smax = p->max_span;
        if (single) {
            const size_t lds = (size_t)lds_private(smax, emax, p->max_intervals, sizeof(Acc));
            if (p->o.atomic_merge) {
                k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
                // numerically symmetric storage (au is al): one value load per entry
                auto kern = private_kernel<VT, YT, kMergeAtomic>(p, al == au);
                if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
                kern<<<p->ntiles, B, lds, s>>>(P, nullptr, A->ia, A->ja, ad, al, au, x, y, smax, emax);
                return hip_status(hipGetLastError());
            } else {
                auto kern = private_kernel<VT, YT, kMergePass>(p, al == au);
                if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
                kern<<<p->ntiles, B, lds, s>>>(P, nullptr, A->ia, A->ja, ad, al, au, x, y, smax, emax);
            }
            if (p->nmerge_blocks > 0 && p->window_slots > 0) {
                if (std::is_same<YT, double>::value)
                    k_merge<Acc, YT, double, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
                else if (p->o.compensated)
                    k_merge<Acc, YT, float, true><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
                else
                    k_merge<Acc, YT, float, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y);
            }
        } else {
            const size_t lds = (size_t)lds_private_mm(smax, emax, p->max_intervals, sizeof(Acc), MmCols<VT>::C);
            if (lds > (size_t)kLdsBudget) return CSRC_ERR_UNSUPPORTED;
            auto kern = k_private_mm<VT, YT>;
            if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
            kern<<<p->ntiles, B, lds, s>>>(P, A->ia, A->ja, ad, al, au, x, ldx, y, ldy, r, smax, emax);
            if (p->nmerge_blocks > 0 && p->window_slots > 0) {
                if (std::is_same<YT, double>::value)
                    k_merge_mm<Acc, YT, double, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y, ldy, r);
                else if (p->o.compensated)
                    k_merge_mm<Acc, YT, float, true><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y, ldy, r);
                else
                    k_merge_mm<Acc, YT, float, false><<<p->nmerge_blocks, kMergeBlock, 0, s>>>(n, P, y, ldy, r);
            }
        }
        break;
    }
    case CSRC_V_OWNER: {
        const int tmax = p->max_tile_rows, pmax = p->max_pull_rows;
        const int emax = std::max(p->max_tile_entries, p->max_pull_entries);
        if (single) {
            const size_t lds = (size_t)lds_owner(tmax, pmax, emax, sizeof(Acc));
            auto kern = k_owner<VT, YT>;
            if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
            kern<<<p->ntiles, B, lds, s>>>(P, A->k, A->ia, A->ja, ad, al, au, x, y, tmax, pmax, emax);
        } else {
            // lanes over the right-hand sides: the plan's lane group covers
            // max_rhs >= r columns
            const int g = p->mm_group;
            const size_t lds = (size_t)lds_owner_pull(tmax, g);
            if (g < 4 || g > 32 || r > g || lds > (size_t)kLdsBudget) return CSRC_ERR_PLAN;
            const void *kern = owner_pull_kernel(A->vdtype, std::is_same<YT, double>::value ? CSRC_F64 : CSRC_F32, g);
            if (!kern) return CSRC_ERR_PLAN;
            if (set_lds(kern, lds)) return CSRC_ERR_HIP;
            void *args[] = {(void *)&P, (void *)&A->ia, (void *)&A->ja, (void *)&ad, (void *)&al, (void *)&au,
                            (void *)&x, (void *)&ldx, (void *)&y, (void *)&ldy, (void *)&r};
            if (hip_status(hipLaunchKernel(kern, dim3(p->ntiles), dim3(B), args, lds, s))) return CSRC_ERR_HIP;
        }
        break;
    }
    case CSRC_V_TILE_COLOR: {
        if (!single) return CSRC_ERR_UNSUPPORTED;
        const int emax = p->max_tile_entries, smax = p->max_span;
        const size_t lds = (size_t)lds_private(smax, emax, p->max_intervals, sizeof(Acc));
        auto kern = private_kernel<VT, YT, kMergeColor>(p, al == au);
        if (set_lds((const void *)kern, lds)) return CSRC_ERR_HIP;
        k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
        // classes in ascending colour order
        for (int cl = 0; cl < p->ncolors; ++cl) {
            const int c0 = p->cptr[cl], c1 = p->cptr[cl + 1];
            kern<<<c1 - c0, B, lds, s>>>(P, P.crow + c0, A->ia, A->ja, ad, al, au, x, y, smax, emax);
        }
        break;
    }
    case CSRC_V_COLOR: {
        k_fill_zero<YT><<<fill_grid((int64_t)n * r), 256, 0, s>>>(y, n, r, ldy);
        for (int c = 0; c < r; ++c)
            for (int cl = 0; cl < p->ncolors; ++cl) {
                const int c0 = p->cptr[cl], c1 = p->cptr[cl + 1];
                const int rows_per_block = (B / G) * kUnroll;
                const int grid = std::max(1, std::min(65535, (c1 - c0 + rows_per_block - 1) / rows_per_block));
                k_color<G, VT, YT><<<grid, B, 0, s>>>(P.crow, c0, c1, A->ia, A->ja, ad, al, au, x + c, ldx, y + c,
                                                      ldy);
            }
        break;
    }
    default:
        return CSRC_ERR_ARG;
    }
    return hip_status(hipGetLastError());
}

template <class VT, class YT>
static int launch_lanes(const csrc_plan *p, const csrc_matrix *A, const void *al, const void *au,
                        const void *x, int64_t ldx, void *y, int64_t ldy, int r, void *ws, hipStream_t s)
{
    switch (p->o.lanes) {
    case 2: return launch_variant<VT, YT, 2>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case 4: return launch_variant<VT, YT, 4>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case 8: return launch_variant<VT, YT, 8>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case 16: return launch_variant<VT, YT, 16>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case 32: return launch_variant<VT, YT, 32>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case 64: return launch_variant<VT, YT, 64>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
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
    // the tile kernels read ja/al/au with 16-byte (8-byte for bfloat16) vector loads
    const uintptr_t va = A->vdtype == CSRC_BF16 ? 8 : 16;
    if (A->k > 0 && (((uintptr_t)A->ja % 16) || ((uintptr_t)A->al % va) || ((uintptr_t)A->au % va)))
        return CSRC_ERR_ARG;
    return CSRC_OK;
}

static int product(const csrc_matrix *A, const csrc_plan *p, int32_t r, const void *x, int64_t ldx,
                   void *y, int64_t ldy, void *ws, int64_t ws_bytes, void *stream, bool transpose)
{
    int st = check_call(A, p, ws, ws_bytes);
    if (st) return st;
    if (r < 1 || r > kMaxRhs || r > p->o.max_rhs || ldx < r || ldy < r) return CSRC_ERR_ARG;
    if (A->n == 0) return CSRC_OK;
    if (!x || !y) return CSRC_ERR_ARG;
    const int ys = (A->vdtype == CSRC_F64 || p->o.ydtype == CSRC_F64) ? 8 : 4;
    const int64_t xspan = ((int64_t)(A->n - 1) * ldx + r) * xbytes(A->vdtype);
    const int64_t yspan = ((int64_t)(A->n - 1) * ldy + r) * ys;
    if (overlap(x, xspan, y, yspan)) return CSRC_ERR_ALIAS;
    const void *al = transpose ? A->au : A->al;
    const void *au = transpose ? A->al : A->au;
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (A->vdtype) {
    case CSRC_F64: return launch_lanes<F64T, double>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case CSRC_F32:
        return p->o.ydtype == CSRC_F64 ? launch_lanes<F32T, double>(p, A, al, au, x, ldx, y, ldy, r, ws, s)
                                       : launch_lanes<F32T, float>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    case CSRC_BF16:
        return p->o.ydtype == CSRC_F64 ? launch_lanes<B16T, double>(p, A, al, au, x, ldx, y, ldy, r, ws, s)
                                       : launch_lanes<B16T, float>(p, A, al, au, x, ldx, y, ldy, r, ws, s);
    default: return CSRC_ERR_ARG;
    }
}

}  // namespace csrc

extern "C" int csrc_spmv(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y,
                         void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, 1, x, 1, y, 1, workspace, ws_bytes, stream, false);
}

extern "C" int csrc_spmv_t(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y,
                           void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, 1, x, 1, y, 1, workspace, ws_bytes, stream, true);
}

extern "C" int csrc_spmm(const csrc_matrix *A, const csrc_plan *plan, int32_t r, const void *X, int64_t ldx,
                         void *Y, int64_t ldy, void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, r, X, ldx, Y, ldy, workspace, ws_bytes, stream, false);
}

extern "C" int csrc_spmm_t(const csrc_matrix *A, const csrc_plan *plan, int32_t r, const void *X, int64_t ldx,
                           void *Y, int64_t ldy, void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::product(A, plan, r, X, ldx, Y, ldy, workspace, ws_bytes, stream, true);
}

// ------------------------------------------------ product without a workspace
//
// For callers that cannot allocate device memory, csrc_spmv_noalloc places
// the plan's tables and its partial buffer in `scratch`, a static device
// array of this source file that each device holds once, for the life of the
// process.  Its device address comes from hipGetSymbolAddress, taken once
// per device with that device current; host code uses only that address.
// Nothing in it needs to start at zero: the plan tables are copied in by
// every call, and every partial slot a merge reads is written first by its
// tile in the same call.  Calls that overlap on one device share the array
// and race.

namespace csrc {

static __device__ __align__(256) unsigned char scratch[CSRC_NOALLOC_MAX_BYTES];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
static int scratch_address(void **out)
{
    int dev = 0;
    int st = hip_status(hipGetDevice(&dev));
    if (st) return st;
    if (dev < 0 || dev >= kMaxDevices) return CSRC_ERR_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (st) return st;
        if (!p) return CSRC_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CSRC_OK;
}

}  // namespace csrc

extern "C" int csrc_spmv_noalloc(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y,
                                 void *stream)
{
    using namespace csrc;
    if (!A || !plan) return CSRC_ERR_ARG;
    if (plan->ws_bytes > (int64_t)CSRC_NOALLOC_MAX_BYTES) return CSRC_ERR_WORKSPACE;
    void *ws = nullptr;
    int st = CSRC_OK;
    if (plan->ws_bytes > 0) {
        st = scratch_address(&ws);
        if (st) return st;
    }
    st = check_call(A, plan, ws, plan->ws_bytes);
    if (st) return st;
    if (A->n == 0) return CSRC_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (plan->blob_bytes > 0) {
        // the plan's host image outlives the call (the caller keeps the plan
        // until the product is done), so the copy is left asynchronous
        st = hip_status(hipMemcpyAsync(ws, plan->blob.data(), (size_t)plan->blob_bytes, hipMemcpyHostToDevice, s));
        if (st) return st;
    }
    return product(A, plan, 1, x, 1, y, 1, ws, plan->ws_bytes, stream, false);
}

namespace csrc {

template <class VT, class YT>
static int launch_pair(const csrc_plan *p, const csrc_matrix *A, const void *x_, void *y_, void *yt_, void *ws,
                       hipStream_t s)
{
    using V = typename VT::V;
    const int32_t n = A->n;
    const int emax = p->max_tile_entries, smax = p->max_span;
    const size_t lds = (size_t)lds_private_pair(smax, emax, p->max_intervals, sizeof(typename VT::A));
    PlanDev P = plan_dev(p, ws);
    YT *y = static_cast<YT *>(y_);
    YT *yt = static_cast<YT *>(yt_);
    auto kern = k_private_pair<VT, YT>;
    if (lds > 65536 && hip_status(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                                      (int)lds)))
        return CSRC_ERR_HIP;
    k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(y, n, 1, 1);
    k_fill_zero<YT><<<fill_grid(n), 256, 0, s>>>(yt, n, 1, 1);
    kern<<<p->ntiles, p->o.block, lds, s>>>(P, A->ia, A->ja, static_cast<const V *>(A->ad),
                                            static_cast<const V *>(A->al), static_cast<const V *>(A->au),
                                            static_cast<const typename VT::X *>(x_), y, yt, smax, emax);
    return hip_status(hipGetLastError());
}

}  // namespace csrc

extern "C" int csrc_spmv_pair(const csrc_matrix *A, const csrc_plan *plan, const void *x, void *y, void *yt,
                              void *workspace, int64_t ws_bytes, void *stream)
{
    using namespace csrc;
    int st = check_call(A, plan, workspace, ws_bytes);
    if (st) return st;
    if (A->n == 0) return CSRC_OK;
    if (!x || !y || !yt) return CSRC_ERR_ARG;
    const int ys = (A->vdtype == CSRC_F64 || plan->o.ydtype == CSRC_F64) ? 8 : 4;
    const int64_t xspan = (int64_t)A->n * xbytes(A->vdtype), yspan = (int64_t)A->n * ys;
    if (overlap(x, xspan, y, yspan) || overlap(x, xspan, yt, yspan) || overlap(y, yspan, yt, yspan))
        return CSRC_ERR_ALIAS;
    const bool fused = plan->o.variant == CSRC_V_PRIVATE && plan->o.atomic_merge &&
                       lds_private_pair(plan->max_span, plan->max_tile_entries, plan->max_intervals,
                                        acc_bytes(A->vdtype)) <= kLdsBudget;
    if (!fused) {
        st = product(A, plan, 1, x, 1, y, 1, workspace, ws_bytes, stream, false);
        return st ? st : product(A, plan, 1, x, 1, yt, 1, workspace, ws_bytes, stream, true);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (A->vdtype) {
    case CSRC_F64: return launch_pair<F64T, double>(plan, A, x, y, yt, workspace, s);
    case CSRC_F32:
        return plan->o.ydtype == CSRC_F64 ? launch_pair<F32T, double>(plan, A, x, y, yt, workspace, s)
                                          : launch_pair<F32T, float>(plan, A, x, y, yt, workspace, s);
    case CSRC_BF16:
        return plan->o.ydtype == CSRC_F64 ? launch_pair<B16T, double>(plan, A, x, y, yt, workspace, s)
                                          : launch_pair<B16T, float>(plan, A, x, y, yt, workspace, s);
    default: return CSRC_ERR_ARG;
    }
}

// ------------------------------------------------------------ rectangular

namespace csrc {

// Rows of A_R (Sec. 2.1, Fig. 2b): y_i += the row's auxiliary CSR entries
// ar x[jar] (rows of A_R are short: one thread per row, no race).
template <class VT, class YT>
__global__ __launch_bounds__(256) void k_rect_gather(int32_t n, const int32_t *__restrict__ iar,
                                                     const int32_t *__restrict__ jar,
                                                     const typename VT::V *__restrict__ ar,
                                                     const typename VT::X *__restrict__ x, YT *__restrict__ y)
{
    using A = typename VT::A;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int q0 = iar[i], q1 = iar[i + 1];
        if (q0 == q1) continue;
        A t = A(0);
        for (int q = q0; q < q1; ++q) t += (A)ldv(ar, q) * (A)x[jar[q]];
        y[i] = y[i] + (YT)t;
    }
}

// Transpose of A_R: every entry (i, jar) adds ar x_i to y[jar] (global
// atomics; y[n, m) is cleared first).
template <class VT, class YT>
__global__ __launch_bounds__(256) void k_rect_scatter(int32_t n, const int32_t *__restrict__ iar,
                                                      const int32_t *__restrict__ jar,
                                                      const typename VT::V *__restrict__ ar,
                                                      const typename VT::X *__restrict__ x, YT *__restrict__ y)
{
    using A = typename VT::A;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int q0 = iar[i], q1 = iar[i + 1];
        if (q0 == q1) continue;
        const A xi = (A)x[i];
        for (int q = q0; q < q1; ++q) atomic_add(&y[jar[q]], (YT)((A)ldv(ar, q) * xi));
    }
}

template <class VT, class YT>
static int launch_rect(const csrc_rect *R, int32_t n, const void *x, void *y, bool transpose, hipStream_t s)
{
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(4096, ((int64_t)n + 255) / 256));
    const auto *ar = static_cast<const typename VT::V *>(R->ar);
    const auto *xv = static_cast<const typename VT::X *>(x);
    YT *yv = static_cast<YT *>(y);
    if (transpose) {
        if (R->m > n) k_fill_zero<YT><<<fill_grid(R->m - n), 256, 0, s>>>(yv + n, R->m - n, 1, 1);
        if (R->kr > 0) k_rect_scatter<VT, YT><<<grid, 256, 0, s>>>(n, R->iar, R->jar, ar, xv, yv);
    } else if (R->kr > 0) {
        k_rect_gather<VT, YT><<<grid, 256, 0, s>>>(n, R->iar, R->jar, ar, xv, yv);
    }
    return hip_status(hipGetLastError());
}

static int rect_product(const csrc_matrix *A, const csrc_rect *R, const csrc_plan *p, const void *x, void *y,
                        void *ws, int64_t ws_bytes, void *stream, bool transpose)
{
    if (!R) return CSRC_ERR_ARG;
    int st = check_call(A, p, ws, ws_bytes);
    if (st) return st;
    if (R->vdtype != A->vdtype || R->m < A->n || R->kr < 0 || (A->n > 0 && !R->iar) ||
        (R->kr > 0 && (!R->jar || !R->ar)))
        return CSRC_ERR_ARG;
    const int32_t n = A->n;
    if (R->m == 0) return CSRC_OK;
    if (!x || !y) return CSRC_ERR_ARG;
    const int ys = (A->vdtype == CSRC_F64 || p->o.ydtype == CSRC_F64) ? 8 : 4;
    const int64_t xn = transpose ? n : R->m, yn = transpose ? R->m : n;
    if (overlap(x, xn * xbytes(A->vdtype), y, yn * ys)) return CSRC_ERR_ALIAS;
    if (n > 0) {
        st = product(A, p, 1, x, 1, y, 1, ws, ws_bytes, stream, transpose);
        if (st) return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    switch (A->vdtype) {
    case CSRC_F64: return launch_rect<F64T, double>(R, n, x, y, transpose, s);
    case CSRC_F32:
        return p->o.ydtype == CSRC_F64 ? launch_rect<F32T, double>(R, n, x, y, transpose, s)
                                       : launch_rect<F32T, float>(R, n, x, y, transpose, s);
    case CSRC_BF16:
        return p->o.ydtype == CSRC_F64 ? launch_rect<B16T, double>(R, n, x, y, transpose, s)
                                       : launch_rect<B16T, float>(R, n, x, y, transpose, s);
    default: return CSRC_ERR_ARG;
    }
}

}  // namespace csrc

extern "C" int csrc_spmv_rect(const csrc_matrix *A, const csrc_rect *R, const csrc_plan *plan, const void *x,
                              void *y, void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::rect_product(A, R, plan, x, y, workspace, ws_bytes, stream, false);
}

extern "C" int csrc_spmv_rect_t(const csrc_matrix *A, const csrc_rect *R, const csrc_plan *plan, const void *x,
                                void *y, void *workspace, int64_t ws_bytes, void *stream)
{
    return csrc::rect_product(A, R, plan, x, y, workspace, ws_bytes, stream, true);
}

// ------------------------------------------------------------ batch launches

namespace csrc {

struct BatchLaunch {
    const void *tiles_fn = nullptr;
    const void *merge_fn = nullptr;   // PRIVATE only
    int grid = 0, merge_grid = 0, block = 512;
    size_t lds = 0;
};

static int device_cus()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

template <class VT, class YT>
static void batch_fns(BatchLaunch &L, bool owner)
{
    using Acc = typename VT::A;
    if (owner) {
        L.tiles_fn = batch_pull_kernel(std::is_same<typename VT::V, double>::value
                                           ? CSRC_F64
                                           : (std::is_same<typename VT::V, float>::value ? CSRC_F32 : CSRC_BF16),
                                       std::is_same<YT, double>::value ? CSRC_F64 : CSRC_F32);
        return;
    }
    L.tiles_fn = (const void *)k_batch_tiles<VT, YT>;
    if (std::is_same<YT, double>::value)
        L.merge_fn = (const void *)k_batch_merge<Acc, YT, double, false>;
    else
        L.merge_fn = (const void *)k_batch_merge<Acc, YT, float, false>;
}

static int batch_launch_config(const csrc_batch_plan *b, BatchLaunch &L)
{
    const bool owner = b->variant == CSRC_V_OWNER;
    switch (b->vdtype) {
    case CSRC_F64: batch_fns<F64T, double>(L, owner); break;
    case CSRC_F32:
        if (b->ydtype == CSRC_F64) batch_fns<F32T, double>(L, owner); else batch_fns<F32T, float>(L, owner);
        break;
    default:
        if (b->ydtype == CSRC_F64) batch_fns<B16T, double>(L, owner); else batch_fns<B16T, float>(L, owner);
    }
    L.block = b->o.block;
    L.lds = (size_t)b->lds;
    const int cus = device_cus();
    const int nitems = (int)(b->items.size() / 2), nm = (int)(b->mitems.size() / 2);
    if (owner) {
        // one workgroup per slot that can be resident (registers, LDS and
        // waves of a CU): each holds a fixed share of its XCD's range, so a
        // workgroup that had to wait for a slot would finish its share late
        if (L.lds > 65536 &&
            hip_status(hipFuncSetAttribute(L.tiles_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds)))
            return CSRC_ERR_HIP;
        int per_cu = 0;
        int st = hip_status(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, L.tiles_fn, L.block, L.lds));
        if (st) return st;
        const int g = b->o.grid > 0 ? b->o.grid : cus * std::max(1, per_cu);
        L.grid = std::max(8, g & ~7);   // a multiple of 8: one share per XCD
        return CSRC_OK;
    } else {
        const int per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(4, kLdsBudget / std::max<int64_t>(1, b->lds)));
        L.grid = b->o.grid > 0 ? b->o.grid : std::max(1, std::min(nitems, cus * per_cu));
        L.merge_grid = std::max(1, std::min(nm, cus * 8));
    }
    if (L.lds > 65536)
        return hip_status(hipFuncSetAttribute(L.tiles_fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds));
    return CSRC_OK;
}

// Kernel arguments of a batch launch (kept alive for the launch or the graph
// node that copies them).
struct BatchArgs {
    const MatDev *mats;
    const int2 *items, *mitems;
    const int32_t *xbeg;
    int nitems, nm, tr, smax, emax;
    void *tiles[6];
    void *merge[3];
    int ntiles_args = 0;

    BatchArgs(const csrc_batch_plan *b, char *ws, int transpose)
    {
        mats = reinterpret_cast<const MatDev *>(ws + b->off_descs);
        items = reinterpret_cast<const int2 *>(ws + b->off_items);
        mitems = reinterpret_cast<const int2 *>(ws + b->off_mitems);
        xbeg = reinterpret_cast<const int32_t *>(ws + b->off_xbeg);
        nitems = (int)(b->items.size() / 2);
        nm = (int)(b->mitems.size() / 2);
        tr = transpose ? 1 : 0;
        smax = b->smax;
        emax = b->emax;
        if (b->variant == CSRC_V_OWNER) {
            // k_batch_pull(mats, items, xbeg, transpose)
            tiles[0] = (void *)&mats;
            tiles[1] = (void *)&items;
            tiles[2] = (void *)&xbeg;
            tiles[3] = (void *)&tr;
            ntiles_args = 4;
        } else {
            // k_batch_tiles(mats, items, nitems, transpose, smax, emax)
            tiles[0] = (void *)&mats;
            tiles[1] = (void *)&items;
            tiles[2] = (void *)&nitems;
            tiles[3] = (void *)&tr;
            tiles[4] = (void *)&smax;
            tiles[5] = (void *)&emax;
            ntiles_args = 6;
        }
        merge[0] = (void *)&mats;
        merge[1] = (void *)&mitems;
        merge[2] = (void *)&nm;
    }
    BatchArgs(const BatchArgs &) = delete;
    BatchArgs &operator=(const BatchArgs &) = delete;
};

}  // namespace csrc

extern "C" int csrc_batch_run(const csrc_batch_plan *b, int32_t transpose, void *workspace, int64_t ws_bytes,
                              void *stream)
{
    using namespace csrc;
    if (!b) return CSRC_ERR_ARG;
    if (!workspace || ws_bytes < b->ws_bytes) return CSRC_ERR_WORKSPACE;
    if (b->items.empty()) return CSRC_OK;
    BatchLaunch L;
    int st = batch_launch_config(b, L);
    if (st) return st;
    BatchArgs a(b, static_cast<char *>(workspace), transpose);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = hip_status(hipLaunchKernel(L.tiles_fn, dim3(L.grid), dim3(L.block), a.tiles, L.lds, s));
    if (st || !L.merge_fn || a.nm == 0) return st;
    return hip_status(hipLaunchKernel(L.merge_fn, dim3(L.merge_grid), dim3(kMergeBlock), a.merge, 0, s));
}

extern "C" int csrc_spmv_batched(const csrc_batch_plan *b, const csrc_matrix *A, const void *const *X,
                                 const int64_t *ldx, void *const *Y, const int64_t *ldy, void *workspace,
                                 int64_t ws_bytes, void *stream)
{
    int st = csrc_batch_bind(b, A, X, ldx, Y, ldy, workspace, ws_bytes, stream);
    return st ? st : csrc_batch_run(b, 0, workspace, ws_bytes, stream);
}

extern "C" int csrc_spmv_t_batched(const csrc_batch_plan *b, const csrc_matrix *A, const void *const *X,
                                   const int64_t *ldx, void *const *Y, const int64_t *ldy, void *workspace,
                                   int64_t ws_bytes, void *stream)
{
    int st = csrc_batch_bind(b, A, X, ldx, Y, ldy, workspace, ws_bytes, stream);
    return st ? st : csrc_batch_run(b, 1, workspace, ws_bytes, stream);
}

extern "C" int csrc_batch_graph_create(const csrc_batch_plan *b, int32_t transpose, void *workspace,
                                       int64_t ws_bytes, csrc_graph **out)
{
    using namespace csrc;
    if (!b || !out) return CSRC_ERR_ARG;
    if (!workspace || ws_bytes < b->ws_bytes) return CSRC_ERR_WORKSPACE;
    *out = nullptr;
    BatchLaunch L;
    int st = batch_launch_config(b, L);
    if (st) return st;
    BatchArgs a(b, static_cast<char *>(workspace), transpose);
    hipGraph_t g = nullptr;
    st = hip_status(hipGraphCreate(&g, 0));
    if (st) return st;
    hipGraphNode_t n1 = nullptr, n2 = nullptr;
    if (a.nitems > 0) {
        hipKernelNodeParams k1{};
        k1.func = const_cast<void *>(L.tiles_fn);
        k1.gridDim = dim3(L.grid);
        k1.blockDim = dim3(L.block);
        k1.sharedMemBytes = (unsigned)L.lds;
        k1.kernelParams = a.tiles;
        st = hip_status(hipGraphAddKernelNode(&n1, g, nullptr, 0, &k1));
        if (!st && L.merge_fn && a.nm > 0) {
            hipKernelNodeParams k2{};
            k2.func = const_cast<void *>(L.merge_fn);
            k2.gridDim = dim3(L.merge_grid);
            k2.blockDim = dim3(kMergeBlock);
            k2.sharedMemBytes = 0;
            k2.kernelParams = a.merge;
            st = hip_status(hipGraphAddKernelNode(&n2, g, &n1, 1, &k2));
        }
    }
    hipGraphExec_t ex = nullptr;
    if (!st) st = hip_status(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
    if (st) {
        hipGraphDestroy(g);
        return st;
    }
    csrc_graph *cg = new (std::nothrow) csrc_graph();
    if (!cg) {
        hipGraphExecDestroy(ex);
        hipGraphDestroy(g);
        return CSRC_ERR_NOMEM;
    }
    cg->graph = g;
    cg->exec = ex;
    *out = cg;
    return CSRC_OK;
}

extern "C" int csrc_graph_launch(csrc_graph *g, void *stream)
{
    if (!g || !g->exec) return CSRC_ERR_ARG;
    return csrc::hip_status(hipGraphLaunch(static_cast<hipGraphExec_t>(g->exec), static_cast<hipStream_t>(stream)));
}

extern "C" int csrc_graph_destroy(csrc_graph *g)
{
    if (!g) return CSRC_OK;
    if (g->exec) (void)hipGraphExecDestroy(static_cast<hipGraphExec_t>(g->exec));
    if (g->graph) (void)hipGraphDestroy(static_cast<hipGraph_t>(g->graph));
    delete g;
    return CSRC_OK;
}

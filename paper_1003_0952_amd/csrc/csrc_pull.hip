// Owner-computes products with several right-hand sides (csrc_spmm and
// csrc_spmm_t with an OWNER plan, and batches of OWNER tiles): the tile
// kernels, and the lookup of their instances for the launch code in
// csrc_spmv.hip.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.h"
#include "internal.h"

namespace csrc {

// --------------------------------------------- OWNER, several right-hand sides
//
// Owner computes with the right-hand sides across lanes: a row's W columns
// (W = 4G >= r, a power of two) are held by a group of G lanes, four columns
// per lane.  Phase 1 gathers each own row in registers,
//     acc = ad_i X[i, :] + sum_{q in row i} al_q X[ja_q, :],
// and stores it into the tile's LDS sums.  Phase 2 walks the tile's pull
// segments -- for every row p at or after the tile, the run of its entries
// whose columns fall into the tile -- and adds au_q X[p, :] to the sums of
// row ja_q with LDS atomics (the column-wise scatter of Fig. 2a, done by the
// owner of the target).  Phase 3 stores the finished rows.  Every Y entry is
// written once: no clearing, no partials, no global atomics, no merge pass.
//
// Memory instructions are what bound this kernel (each touches several
// cache lines), so they are made wide: a lane reads its part of an x row as
// 16-byte pieces -- FP64: columns {2c, 2c+1} and {W/2 + 2c, W/2 + 2c + 1},
// so a group's first piece is one contiguous run of W/2 values; FP32: the
// four columns 4c..4c+3 -- and a row's entries four at a time (ja as 16
// bytes, FP64 values as 2 x 16, FP32 as 16).  A piece that would reach past
// the last column, or a group of entries past the row's end, is read value
// by value instead, so no load leaves its row or its array.

typedef double d2u __attribute__((ext_vector_type(2), aligned(8)));
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef int i4u __attribute__((ext_vector_type(4), aligned(4)));

// Four entries from q (entries from qe on are absent: j = -1, value 0):
// column indices and values of vals, as the accumulator type.
template <class VT>
__device__ __forceinline__ void entries4(const int32_t *__restrict__ ja, const typename VT::V *__restrict__ vals,
                                         int q, int qe, int (&j)[4], typename VT::A (&a)[4])
{
    using V = typename VT::V;
    using A = typename VT::A;
    if (q + 3 < qe) {
        const i4u jj = *reinterpret_cast<const i4u *>(ja + q);
        j[0] = jj.x;
        j[1] = jj.y;
        j[2] = jj.z;
        j[3] = jj.w;
        if constexpr (std::is_same<V, double>::value) {
            const d2u v0 = *reinterpret_cast<const d2u *>(vals + q);
            const d2u v1 = *reinterpret_cast<const d2u *>(vals + q + 2);
            a[0] = v0.x;
            a[1] = v0.y;
            a[2] = v1.x;
            a[3] = v1.y;
        } else if constexpr (std::is_same<V, float>::value) {
            const f4u v = *reinterpret_cast<const f4u *>(vals + q);
            a[0] = v.x;
            a[1] = v.y;
            a[2] = v.z;
            a[3] = v.w;
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) a[u] = (A)ldv(vals, q + u);
        }
        return;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const bool ok = q + u < qe;
        j[u] = ok ? ja[q + u] : -1;
        a[u] = ok ? (A)ldv(vals, q + u) : A(0);
    }
}

// One owner tile t with r columns (r <= 4G).  s_y: LDS, rows x owner_mm_ld(4G)
// FP64 sums.  Called by every thread of the workgroup.
template <class VT, class YT, int G>
__device__ __forceinline__ void owner_tile_pull(const PlanDev &P, int t, const int32_t *__restrict__ ia,
                                                const int32_t *__restrict__ ja,
                                                const typename VT::V *__restrict__ ad,
                                                const typename VT::V *__restrict__ al,
                                                const typename VT::V *__restrict__ au,
                                                const typename VT::X *__restrict__ X, int64_t ldx,
                                                YT *__restrict__ Y, int64_t ldy, int r, double *s_y)
{
    using A = typename VT::A;
    using Xt = typename VT::X;
    constexpr int W = 4 * G;                  // columns per row
    constexpr int LD = owner_mm_ld(W);
    constexpr bool kX64 = sizeof(Xt) == 8;
    static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "lane group");
    const int tid = threadIdx.x, lane = tid & 63;
    const int lc = lane & (G - 1);
    const int grp = tid / G, ngrp = (int)blockDim.x / G;
    int col[4];                               // the columns this lane holds
#pragma unroll
    for (int v = 0; v < 4; ++v) col[v] = kX64 ? (v >> 1) * (W / 2) + 2 * lc + (v & 1) : 4 * lc + v;
    const int r0 = P.tiles[t], r1 = P.tiles[t + 1], T = r1 - r0;
    auto xrow = [&](int row, A(&o)[4]) {
        const Xt *p = X + (int64_t)row * ldx;
        if constexpr (kX64) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int b = col[2 * h];
                if (b + 1 < r) {
                    const d2u v = *reinterpret_cast<const d2u *>(p + b);
                    o[2 * h] = v.x;
                    o[2 * h + 1] = v.y;
                } else {
                    o[2 * h] = b < r ? (A)p[b] : A(0);
                    o[2 * h + 1] = A(0);
                }
            }
        } else {
            const int b = col[0];
            if (b + 3 < r) {
                const f4u v = *reinterpret_cast<const f4u *>(p + b);
                o[0] = v.x;
                o[1] = v.y;
                o[2] = v.z;
                o[3] = v.w;
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) o[v] = b + v < r ? (A)p[b + v] : A(0);
            }
        }
    };
    __syncthreads();   // the workgroup's previous tile has left the LDS

    // phase 1: own rows, row-wise gather in registers; the next four
    // entries load while the current four's x rows do
    for (int i = grp; i < T; i += ngrp) {
        const int row = r0 + i;
        const int q0 = ia[row], q1 = ia[row + 1];
        A acc[4];
        {
            A xi[4];
            xrow(row, xi);
            const A d = (A)ldv(ad, row);
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = d * xi[v];
        }
        int jn[4];
        A an[4];
        entries4<VT>(ja, al, q0, q1, jn, an);
        for (int qb = q0; qb < q1; qb += 4) {
            int jc[4];
            A ac[4], xv[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                jc[u] = jn[u];
                ac[u] = an[u];
                if (jc[u] >= 0) {
                    xrow(jc[u], xv[u]);
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) xv[u][v] = A(0);
                }
            }
            if (qb + 4 < q1) entries4<VT>(ja, al, qb + 4, q1, jn, an);
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[v] += ac[u] * xv[u][v];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v)
            if (col[v] < r) s_y[i * LD + col[v]] = (double)acc[v];
    }
    __syncthreads();

    // phase 2: the scatters into the tile, pulled from the rows that make them
    const int s0 = P.seg_ptr[t], s1 = P.seg_ptr[t + 1];
    for (int g = s0 + grp; g < s1; g += ngrp) {
        const PullSeg sg = P.segs[g];
        A xp[4];
        xrow(sg.row, xp);
        for (int qb = sg.q0; qb < sg.q1; qb += 4) {
            int jc[4];
            A uc[4];
            entries4<VT>(ja, au, qb, sg.q1, jc, uc);
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (jc[u] >= 0) {
                    const int base = (jc[u] - r0) * LD;
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        if (col[v] < r) atomic_add(&s_y[base + col[v]], (double)(uc[u] * xp[v]));
                }
        }
    }
    __syncthreads();

    // phase 3: the finished rows (consecutive threads on consecutive columns)
    for (int e = tid; e < T * W; e += blockDim.x) {
        const int i = e / W, cc = e % W;
        if (cc < r) Y[(int64_t)(r0 + i) * ldy + cc] = (YT)s_y[i * LD + cc];
    }
}

// Waves per SIMD the owner multi-column kernels are compiled for: the
// kernels wait on memory most of the time and need every wave, so eight
// (64 VGPRs) for FP32 and BF16 values; six for FP64 (at most 85 VGPRs: 64
// would spill).
template <class VT> struct PullWaves { static constexpr int value = 8; };
template <> struct PullWaves<F64T> { static constexpr int value = 6; };

template <class VT, class YT, int G>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(PullWaves<VT>::value))) void k_owner_pull(PlanDev P, const int32_t *__restrict__ ia,
                                                    const int32_t *__restrict__ ja,
                                                    const typename VT::V *__restrict__ ad,
                                                    const typename VT::V *__restrict__ al,
                                                    const typename VT::V *__restrict__ au,
                                                    const typename VT::X *__restrict__ X, int64_t ldx,
                                                    YT *__restrict__ Y, int64_t ldy, int r)
{
    extern __shared__ __align__(16) unsigned char lds[];
    owner_tile_pull<VT, YT, G>(P, xcd_tile(blockIdx.x, gridDim.x), ia, ja, ad, al, au, X, ldx, Y, ldy, r,
                               reinterpret_cast<double *>(lds));
}

// Batched owner products: the work list holds (matrix, tile) items in matrix
// order, cut into 8 ranges of equal cost (xbeg[0..8]); the workgroups of XCD x
// (blockIdx mod 8) walk range x with a stride, so neighbouring tiles of one
// matrix share that XCD's L2.  The grid is a multiple of 8.
template <class VT, class YT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(PullWaves<VT>::value))) void k_batch_pull(const MatDev *__restrict__ mats, const int2 *__restrict__ items,
                                                    const int32_t *__restrict__ xbeg, int transpose)
{
    extern __shared__ __align__(16) unsigned char lds[];
    using V = typename VT::V;
    using Xt = typename VT::X;
    double *s_y = reinterpret_cast<double *>(lds);
    const int x = blockIdx.x & 7, per = gridDim.x >> 3;
    const int e1 = xbeg[x + 1];
    for (int it = xbeg[x] + (int)(blockIdx.x >> 3); it < e1; it += per) {
        const int2 w = items[it];
        const MatDev &M = mats[w.x];
        const V *al = static_cast<const V *>(transpose ? M.au : M.al);
        const V *au = static_cast<const V *>(transpose ? M.al : M.au);
        const V *ad = static_cast<const V *>(M.ad);
        const Xt *Xm = static_cast<const Xt *>(M.X);
        YT *Ym = static_cast<YT *>(M.Y);
        // M.g columns per row (4..32): groups of M.g / 4 lanes
        switch (M.g) {
        case 4: owner_tile_pull<VT, YT, 1>(M.P, w.y, M.ia, M.ja, ad, al, au, Xm, M.ldx, Ym, M.ldy, M.r, s_y); break;
        case 8: owner_tile_pull<VT, YT, 2>(M.P, w.y, M.ia, M.ja, ad, al, au, Xm, M.ldx, Ym, M.ldy, M.r, s_y); break;
        case 16: owner_tile_pull<VT, YT, 4>(M.P, w.y, M.ia, M.ja, ad, al, au, Xm, M.ldx, Ym, M.ldy, M.r, s_y); break;
        default: owner_tile_pull<VT, YT, 8>(M.P, w.y, M.ia, M.ja, ad, al, au, Xm, M.ldx, Ym, M.ldy, M.r, s_y); break;
        }
    }
}

// Kernel instances for the launch code.
template <class VT, class YT>
static const void *owner_pull_for(int w)
{
    switch (w) {
    case 4: return (const void *)k_owner_pull<VT, YT, 1>;
    case 8: return (const void *)k_owner_pull<VT, YT, 2>;
    case 16: return (const void *)k_owner_pull<VT, YT, 4>;
    case 32: return (const void *)k_owner_pull<VT, YT, 8>;
    default: return nullptr;
    }
}

const void *owner_pull_kernel(int32_t vdtype, int32_t ydtype, int w)
{
    const bool y64 = ydtype == CSRC_F64;
    switch (vdtype) {
    case CSRC_F64: return owner_pull_for<F64T, double>(w);
    case CSRC_F32: return y64 ? owner_pull_for<F32T, double>(w) : owner_pull_for<F32T, float>(w);
    case CSRC_BF16: return y64 ? owner_pull_for<B16T, double>(w) : owner_pull_for<B16T, float>(w);
    default: return nullptr;
    }
}

const void *batch_pull_kernel(int32_t vdtype, int32_t ydtype)
{
    const bool y64 = ydtype == CSRC_F64;
    switch (vdtype) {
    case CSRC_F64: return (const void *)k_batch_pull<F64T, double>;
    case CSRC_F32: return y64 ? (const void *)k_batch_pull<F32T, double> : (const void *)k_batch_pull<F32T, float>;
    case CSRC_BF16: return y64 ? (const void *)k_batch_pull<B16T, double> : (const void *)k_batch_pull<B16T, float>;
    default: return nullptr;
    }
}

}  // namespace csrc

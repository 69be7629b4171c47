// Device helpers shared by the libcsrc kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace csrc {

// ---- value types --------------------------------------------------------
// Storage V, source-vector X and accumulator A types per storage dtype, and
// S, the type of the LDS sums that take scattered adds:
//   F64 storage: double / double / double, sums double
//   F32 storage: float  / float  / float,  sums double
//   BF16 storage: uint16 (bfloat16 bits) / float / float, sums double
// Products, row sums, partials and the merge use A; only the LDS sums are
// FP64 for every storage type, because the LDS of gfx950 executes ds_add_f64
// at about twenty times the rate of ds_add_f32.
struct F64T { using V = double;   using X = double; using A = double; using S = double; static constexpr bool kSym = false; };
struct F32T { using V = float;    using X = float;  using A = float;  using S = double; static constexpr bool kSym = false; };
struct B16T { using V = uint16_t; using X = float;  using A = float;  using S = double; static constexpr bool kSym = false; };
// Numerically symmetric storage of a value type: au is al, so the value of
// an entry is loaded once and serves both the gather and the scatter.
template <class Base>
struct SymT : Base { static constexpr bool kSym = true; };

__device__ __forceinline__ double ldv(const double *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const float *p, int64_t i) { return p[i]; }
__device__ __forceinline__ float ldv(const uint16_t *p, int64_t i)
{
    return __uint_as_float(((uint32_t)p[i]) << 16);
}

// Hardware floating-point atomic add (global_atomic_add_f64/f32 on device
// memory, ds_add_f64/f32 on LDS).  Return value unused.
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }

// Sum over the g lanes of an aligned lane group (g a power of two <= 64);
// every lane of the group receives the total.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v)
{
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// Workgroups are dispatched to the 8 XCDs round robin (workgroup b runs on
// XCD b mod 8).  Map b to a tile so that each XCD owns one contiguous range
// of tiles: neighbouring tiles then share that XCD's L2.  Bijective for any
// grid size.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    constexpr int X = 8;
    int q = nb / X, rem = nb % X;
    int x = b % X, j = b / X;
    return x * q + (x < rem ? x : rem) + j;
}

}  // namespace csrc

// Device helpers shared by the libcsrc kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace csrc {

// ---- value types --------------------------------------------------------
// Storage V, source-vector X and accumulator A types per storage dtype:
//   F64 storage: double / double / double
//   F32 storage: float  / float  / float
//   BF16 storage: uint16 (bfloat16 bits) / float / float
struct F64T { using V = double;   using X = double; using A = double; };
struct F32T { using V = float;    using X = float;  using A = float;  };
struct B16T { using V = uint16_t; using X = float;  using A = float;  };

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

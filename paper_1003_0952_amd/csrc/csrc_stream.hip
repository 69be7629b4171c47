// Streaming probes of the HBM ceiling: the rate at which one kernel can read
// (or copy) a large buffer on this device.  They bound what the products can
// reach -- every product is an HBM read stream with a small write side -- and
// are reported beside them; they compute nothing of the method.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace csrc {

typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// Workgroup b of the grid handles one contiguous run of the `count`
// 16-byte words: [b * per, min(count, (b + 1) * per)).  A contiguous run per
// workgroup reads about a seventh faster on this device than a grid-stride
// walk over the same bytes (HBM row locality), so the probes measure that.
__device__ __forceinline__ void chunk_of(int64_t count, int64_t &b, int64_t &e)
{
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    b = blockIdx.x * per;
    e = min(count, b + per);
}

// Read `count` 16-byte words with non-temporal loads, four in flight per
// thread per step; each workgroup writes the xor of everything it read to
// sink[blockIdx.x] so that no load is dead.
__global__ __launch_bounds__(256) void k_stream_read(const u4v *__restrict__ src, int64_t count,
                                                     uint32_t *__restrict__ sink)
{
    constexpr int U = 4;
    const int B = blockDim.x;
    int64_t b, e;
    chunk_of(count, b, e);
    int64_t i = b + threadIdx.x;
    u4v acc = {0u, 0u, 0u, 0u};
    for (; i + (U - 1) * B < e; i += U * B) {
        u4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * B);
#pragma unroll
        for (int u = 0; u < U; ++u) acc ^= v[u];
    }
    for (; i < e; i += B) acc ^= __builtin_nontemporal_load(src + i);
    uint32_t w = acc.x ^ acc.y ^ acc.z ^ acc.w;
    for (int off = 32; off > 0; off >>= 1) w ^= __shfl_xor(w, off);
    __shared__ uint32_t red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t ^= red[k];
        sink[blockIdx.x] = t;
    }
}

// Copy `count` 16-byte words (non-temporal loads and stores), one contiguous
// run per workgroup.
__global__ __launch_bounds__(256) void k_stream_copy(const u4v *__restrict__ src, u4v *__restrict__ dst,
                                                     int64_t count)
{
    constexpr int U = 4;
    const int B = blockDim.x;
    int64_t b, e;
    chunk_of(count, b, e);
    int64_t i = b + threadIdx.x;
    for (; i + (U - 1) * B < e; i += U * B) {
        u4v v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + i + u * B);
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u], dst + i + u * B);
    }
    for (; i < e; i += B) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace csrc

extern "C" int csrc_stream_read(const void *src, int64_t bytes, uint32_t *sink, int32_t grid, void *stream)
{
    if (!src || !sink || bytes < 0 || (bytes & 15) || grid < 1 || grid > 65536) return CSRC_ERR_ARG;
    if (((uintptr_t)src & 15) || ((uintptr_t)sink & 3)) return CSRC_ERR_ARG;
    if (bytes == 0) return CSRC_OK;
    csrc::k_stream_read<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const csrc::u4v *>(src), bytes / 16, sink);
    return csrc::hip_status(hipGetLastError());
}

extern "C" int csrc_stream_copy(const void *src, void *dst, int64_t bytes, int32_t grid, void *stream)
{
    if (!src || !dst || bytes < 0 || (bytes & 15) || grid < 1 || grid > 65536) return CSRC_ERR_ARG;
    if (((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return CSRC_ERR_ARG;
    const char *s = static_cast<const char *>(src);
    const char *d = static_cast<const char *>(dst);
    if (s < d + bytes && d < s + bytes) return CSRC_ERR_ALIAS;
    if (bytes == 0) return CSRC_OK;
    csrc::k_stream_copy<<<grid, 256, 0, static_cast<hipStream_t>(stream)>>>(
        static_cast<const csrc::u4v *>(src), static_cast<csrc::u4v *>(dst), bytes / 16);
    return csrc::hip_status(hipGetLastError());
}

// Epoch-write and interest-vector kernels.
//
// Epoch writes (section "Evaluation", cost of operations: writes go to the
// DRAM working copy and a snapshot is periodically copied into the GPU): the
// staged buckets are scattered into the back copy of the database, and after
// the swap the same buckets are copied into the new back copy.
//
// Interest vector (section "Private Notifications"): each write ORs its
// interest-vector bits into the open epoch's delta; the published global
// vector is the OR of the last `window` deltas.
#include <hip/hip_runtime.h>

#include "engine.h"

namespace talek {
namespace {

constexpr int WG = 256;

// One workgroup per row; rows are `stride16` uint4 long.
__global__ __launch_bounds__(WG) void scatter_rows_kernel(uint4 *__restrict__ dst, const uint4 *__restrict__ src,
                                                          const uint64_t *__restrict__ idx, uint64_t stride16,
                                                          bool src_indexed)
{
    const uint64_t e = blockIdx.x;
    const uint64_t row = idx[e];
    const uint4 *s = src + (src_indexed ? row : e) * stride16;
    uint4 *d = dst + row * stride16;
    for (uint64_t c = threadIdx.x; c < stride16; c += WG)
        d[c] = s[c];
}

__global__ __launch_bounds__(WG) void fill_zero_kernel(uint32_t *__restrict__ p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < words; i += (uint64_t)gridDim.x * WG)
        p[i] = 0u;
}

// bit p lives in word p >> 5, bit p & 31 (little-endian: byte p >> 3, bit p & 7)
__global__ __launch_bounds__(WG) void set_bits_kernel(uint32_t *__restrict__ words, const uint32_t *__restrict__ pos,
                                                      uint64_t count)
{
    const uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= count)
        return;
    const uint32_t p = pos[i];
    atomicOr(words + (p >> 5), 1u << (p & 31u));
}

__global__ __launch_bounds__(WG) void or_rows_kernel(uint32_t *__restrict__ out, const uint32_t *__restrict__ rows,
                                                     uint32_t nrows, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < words; i += (uint64_t)gridDim.x * WG) {
        uint32_t v = 0;
        for (uint32_t r = 0; r < nrows; ++r)
            v |= rows[(uint64_t)r * words + i];
        out[i] = v;
    }
}

uint32_t grid_for(uint64_t items)
{
    uint64_t g = (items + WG - 1) / WG;
    if (g > 65536)
        g = 65536;
    return (uint32_t)(g ? g : 1);
}

}  // namespace

hipError_t launch_scatter_rows(void *dst, const void *src, const uint64_t *idx, uint64_t count, uint64_t stride,
                               hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((uint32_t)count), dim3(WG), 0, stream, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), idx, stride / 16, false);
    return hipGetLastError();
}

hipError_t launch_copy_rows(void *dst, const void *src, const uint64_t *idx, uint64_t count, uint64_t stride,
                            hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(scatter_rows_kernel, dim3((uint32_t)count), dim3(WG), 0, stream, static_cast<uint4 *>(dst),
                       static_cast<const uint4 *>(src), idx, stride / 16, true);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, uint64_t bytes, hipStream_t stream)
{
    const uint64_t words = bytes / 4;
    if (words == 0)
        return hipSuccess;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(grid_for(words)), dim3(WG), 0, stream, static_cast<uint32_t *>(p),
                       words);
    return hipGetLastError();
}

hipError_t launch_set_bits(uint32_t *words, const uint32_t *pos, uint64_t count, hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(set_bits_kernel, dim3((uint32_t)((count + WG - 1) / WG)), dim3(WG), 0, stream, words, pos,
                       count);
    return hipGetLastError();
}

hipError_t launch_or_rows(uint32_t *out, const uint32_t *rows, uint32_t nrows, uint64_t words, hipStream_t stream)
{
    if (words == 0)
        return hipSuccess;
    hipLaunchKernelGGL(or_rows_kernel, dim3(grid_for(words)), dim3(WG), 0, stream, out, rows, nrows, words);
    return hipGetLastError();
}

}  // namespace talek

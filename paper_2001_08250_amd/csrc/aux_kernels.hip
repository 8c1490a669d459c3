// Epoch-write and interest-vector kernels.
//
// Epoch writes (section "Evaluation", cost of operations: writes go to the
// DRAM working copy and a snapshot is periodically copied into the GPU): the
// staged buckets are scattered into the back copy of the database, and after
// the swap the same buckets are copied into the new back copy.
//
// Interest vector (section "Private Notifications"): the writes of an epoch
// OR their interest-vector bits into that epoch's delta; the published global
// vector is the OR of the last `window` deltas. Both are built by the commit
// kernel, in the same launch that applies the staged bucket rows.
#include <hip/hip_runtime.h>

#include <algorithm>

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
// The device half of an epoch commit, one launch. Blocks below iv_blocks
// each own COMMIT_IV_WORDS words of the interest vector: they OR the window's other
// slots, build the new epoch's delta from the positions that fall into their
// words (the host sorted them by block), store the delta in its ring slot
// (overwriting the epoch that leaves the window) and write the new global
// vector. The remaining blocks copy one staged bucket row each (read in
// place from mapped host memory) into the back copy.
__global__ __launch_bounds__(WG) void commit_kernel(const CommitArgs a)
{
    const uint64_t b = blockIdx.x;
    if (b >= a.iv_blocks) {
        const uint64_t e = b - a.iv_blocks;
        const uint64_t row = a.idx[e];
        const uint4 *s = a.rows + e * a.stride16;
        uint4 *d = a.back + row * a.stride16;
        for (uint64_t c = threadIdx.x; c < a.stride16; c += WG)
            d[c] = s[c];
        return;
    }
    constexpr uint32_t W = COMMIT_IV_WORDS, SL = WG / COMMIT_IV_WORDS;
    __shared__ uint32_t part[SL][W];
    __shared__ uint32_t fresh[W];
    const uint32_t lane = threadIdx.x % W, sl = threadIdx.x / W;
    const uint64_t i = b * W + lane;
    if (threadIdx.x < W)
        fresh[threadIdx.x] = 0u;
    uint32_t v = 0;
    if (i < a.words) {
#pragma unroll 8
        for (uint32_t r = sl; r < a.window; r += SL)
            if (r != a.slot)
                v |= a.ring[(uint64_t)r * a.words + i];
    }
    part[sl][lane] = v;
    __syncthreads();
    for (uint32_t j = a.pos_start[b] + threadIdx.x; j < a.pos_start[b + 1]; j += WG) {
        const uint32_t p = a.pos[j];
        const uint64_t w = (uint64_t)(p >> 5) - b * W;
        if (w < W)
            atomicOr(&fresh[w], 1u << (p & 31u));
    }
    __syncthreads();
    if (sl == 0 && i < a.words) {
        uint32_t o = fresh[lane];
        a.ring[(uint64_t)a.slot * a.words + i] = o;
#pragma unroll
        for (uint32_t k = 0; k < SL; ++k)
            o |= part[k][lane];
        a.global[i] = o;
    }
}

// Request staging: Qt[w][r] = word w of request row r (bits >= n cleared),
// rows r in [B, Bp) zero. 64 x 64 word tiles transposed through LDS so both
// the reads (along a row) and the writes (along a word column) coalesce.
__global__ __launch_bounds__(WG) void transpose_requests_kernel(const uint32_t *__restrict__ Q, uint64_t qpitch_w,
                                                                uint32_t B, uint64_t n, uint32_t *__restrict__ Qt,
                                                                uint32_t Bp)
{
    __shared__ uint32_t tile[64][65];
    const uint64_t nwords = (n + 31) >> 5;
    const uint64_t w0 = (uint64_t)blockIdx.x * 64;
    const uint32_t r0 = blockIdx.y * 64;
    const uint32_t tx = threadIdx.x & 63u, ty = threadIdx.x >> 6;
    for (uint32_t i = ty; i < 64; i += WG / 64) {
        const uint32_t r = r0 + i;
        const uint64_t w = w0 + tx;
        uint32_t v = 0;
        if (r < B && w < nwords) {
            v = Q[(uint64_t)r * qpitch_w + w];
            if (((w + 1) << 5) > n)
                v &= (1u << (n & 31u)) - 1u;
        }
        tile[i][tx] = v;
    }
    __syncthreads();
    for (uint32_t i = ty; i < 64; i += WG / 64) {
        const uint64_t w = w0 + i;
        const uint32_t r = r0 + tx;
        if (w < nwords && r < Bp)
            Qt[w * Bp + r] = tile[tx][i];
    }
}

// Four-Russians staging: Qs[g * Bp + r] = (byte g of request row r) << 8,
// i.e. the LDS byte offset of that request's table entry for bucket group g
// (bits >= n cleared, rows B <= r < Bp zero).
__global__ __launch_bounds__(WG) void stage_group_offsets_kernel(const uint32_t *__restrict__ Q, uint64_t qpitch_w,
                                                                 uint32_t B, uint64_t n, uint32_t *__restrict__ Qs,
                                                                 uint32_t Bp)
{
    __shared__ uint32_t tile[64][65];
    const uint64_t nwords = (n + 31) >> 5;
    const uint64_t w0 = (uint64_t)blockIdx.x * 64;
    const uint32_t r0 = blockIdx.y * 64;
    const uint32_t tx = threadIdx.x & 63u, ty = threadIdx.x >> 6;
    for (uint32_t i = ty; i < 64; i += WG / 64) {
        const uint32_t r = r0 + i;
        const uint64_t w = w0 + tx;
        uint32_t v = 0;
        if (r < B && w < nwords) {
            v = Q[(uint64_t)r * qpitch_w + w];
            if (((w + 1) << 5) > n)
                v &= (1u << (n & 31u)) - 1u;
        }
        tile[i][tx] = v;
    }
    __syncthreads();
    for (uint32_t i = ty; i < 64; i += WG / 64) {
        const uint64_t w = w0 + i;
        const uint32_t r = r0 + tx;
        if (w < nwords && r < Bp) {
            const uint32_t v = tile[tx][i];
#pragma unroll
            for (uint32_t k = 0; k < 4; ++k)
                Qs[(w * 4 + k) * Bp + r] = ((v >> (8 * k)) & 0xffu) << 8;
        }
    }
}

// dst row i = src row rows[i] for i < count (row16 uint4 per row). Used by
// the serving loop to pull the request rows of a batch straight out of
// pinned host memory (src and rows are host-mapped).
__global__ __launch_bounds__(WG) void gather_rows_kernel(uint4 *__restrict__ dst, uint64_t dst_pitch16,
                                                         const uint4 *__restrict__ src, uint64_t src_pitch16,
                                                         const uint32_t *__restrict__ rows, uint32_t row16)
{
    const uint64_t i = blockIdx.x;
    const uint4 *s = src + (uint64_t)rows[i] * src_pitch16;
    uint4 *d = dst + i * dst_pitch16;
    for (uint32_t c = threadIdx.x; c < row16; c += WG)
        d[c] = s[c];
}

// dst row (dst_rows ? dst_rows[i] : i) = src row (src_rows ? src_rows[i] : i),
// row_w 32-bit words per row; workgroup i copies row i.
__global__ __launch_bounds__(WG) void move_rows_kernel(uint32_t *__restrict__ dst, uint64_t dst_pitch_w,
                                                       const uint64_t *__restrict__ dst_rows,
                                                       const uint32_t *__restrict__ src, uint64_t src_pitch_w,
                                                       const uint64_t *__restrict__ src_rows, uint64_t row_w)
{
    const uint64_t i = blockIdx.x;
    const uint32_t *s = src + (src_rows ? src_rows[i] : i) * src_pitch_w;
    uint32_t *d = dst + (dst_rows ? dst_rows[i] : i) * dst_pitch_w;
    for (uint64_t c = threadIdx.x; c < row_w; c += WG)
        d[c] = s[c];
}

uint32_t grid_for(uint64_t items)
{
    uint64_t g = (items + WG - 1) / WG;
    if (g > 65536)
        g = 65536;
    return (uint32_t)(g ? g : 1);
}

}  // namespace

hipError_t launch_move_rows(void *dst, uint64_t dst_pitch, const uint64_t *dst_rows, const void *src,
                            uint64_t src_pitch, const uint64_t *src_rows, uint64_t count, uint64_t row_bytes,
                            hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    if (count > 0x7fffffffull || (dst_pitch & 3) || (src_pitch & 3) || (row_bytes & 3))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(move_rows_kernel, dim3((uint32_t)count), dim3(WG), 0, stream, static_cast<uint32_t *>(dst),
                       dst_pitch / 4, dst_rows, static_cast<const uint32_t *>(src), src_pitch / 4, src_rows,
                       row_bytes / 4);
    return hipGetLastError();
}

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

hipError_t launch_transpose_requests(const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t *Qt,
                                     uint32_t Bp, hipStream_t stream)
{
    const uint64_t nwords = (n + 31) / 32;
    if (nwords == 0 || Bp == 0)
        return hipSuccess;
    dim3 grid((uint32_t)((nwords + 63) / 64), (Bp + 63) / 64);
    hipLaunchKernelGGL(transpose_requests_kernel, grid, dim3(WG), 0, stream, static_cast<const uint32_t *>(Q),
                       qpitch / 4, B, n, Qt, Bp);
    return hipGetLastError();
}

hipError_t launch_stage_group_offsets(const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t *Qs,
                                      uint32_t Bp, hipStream_t stream)
{
    const uint64_t nwords = (n + 31) / 32;
    if (nwords == 0 || Bp == 0)
        return hipSuccess;
    dim3 grid((uint32_t)((nwords + 63) / 64), (Bp + 63) / 64);
    hipLaunchKernelGGL(stage_group_offsets_kernel, grid, dim3(WG), 0, stream, static_cast<const uint32_t *>(Q),
                       qpitch / 4, B, n, Qs, Bp);
    return hipGetLastError();
}

hipError_t launch_gather_rows(void *dst, uint64_t dst_pitch, const void *src, uint64_t src_pitch,
                              const uint32_t *rows, uint32_t count, uint64_t row_bytes, hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(count), dim3(WG), 0, stream, static_cast<uint4 *>(dst),
                       dst_pitch / 16, static_cast<const uint4 *>(src), src_pitch / 16, rows,
                       (uint32_t)((row_bytes + 15) / 16));
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

hipError_t launch_commit(const CommitArgs &a, hipStream_t stream)
{
    const uint64_t blocks = a.iv_blocks + a.nrows;
    if (blocks == 0)
        return hipSuccess;
    if (blocks > 0x7fffffffull)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(commit_kernel, dim3((uint32_t)blocks), dim3(WG), 0, stream, a);
    return hipGetLastError();
}

}  // namespace talek

// XOR-PIR read kernels for gfx950: tiled masked / zero-skip families and the
// split-partial reduction.
//
// The server answer (section "Background: PIR", server step) is the GF(2)
// product of the request bit matrix R (B x n) with the database D (n buckets
// of `stride` bytes): resp[r] = XOR over j with R[r][j] = 1 of D[j].
//
// Mapping on CDNA4 (wave64):
//  * A workgroup is 4 waves. Each lane owns 16 bytes of a bucket row, so one
//    wave covers a 1 KiB column chunk and a workgroup a 4 KiB column group.
//    Loads of D are 16 B per lane, fully coalesced (global_load_dwordx4).
//  * A wave accumulates T requests ("tile") in VGPRs: acc[T] x 4 dwords.
//  * Request bits are wave-uniform (every lane of the wave works on the same
//    bucket), so the 32-bit request words are fetched with scalar loads and
//    every per-(request, bucket) decision lives on the SALU.
//  * MASK family: acc ^= data & mask, one v_bitop3_b32 per dword (truth table
//    0x78 = S0 ^ (S1 & S2)) with the 0 / ~0 mask built on the SALU.
//  * SKIP family: a wave-uniform branch skips unselected buckets, so only
//    selected buckets cost a v_xor (half of them for uniform requests).
//  * Buckets are split into `splits` contiguous ranges (multiples of 32
//    buckets); each split writes a partial answer and a second pass XORs the
//    partials (XOR is associative and commutative, so this is exact).
//  * Work decomposition is XCD-aware: workgroups are dispatched round-robin
//    over the 8 XCDs, so task t is given to blockIdx (t % per) * 8 + t / per
//    with request tiles fastest. The request tiles that share a (split,
//    column group) slice of D then run together on one XCD and reuse it from
//    that XCD's L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace talek {
namespace {

constexpr int WG = 256;
constexpr uint32_t COLS_PER_WG = 4 * 64;  // uint4 columns per workgroup (4 KiB)

struct TileArgs {
    const uint4 *D;
    uint64_t n;
    uint32_t stride16;
    uint32_t B;
    const uint32_t *Q;
    uint64_t qpitch_w;
    uint4 *out;
    uint64_t out_row16;
    uint64_t out_split16;
    uint32_t n_rt, n_cg, splits, words_per_split, tasks_per_xcd;
};

__device__ __forceinline__ uint32_t xor_and(uint32_t acc, uint32_t v, uint32_t m)
{
    return __builtin_amdgcn_bitop3_b32(acc, v, m, 0x78);  // acc ^ (v & m)
}

template <int T, int KIND>
__device__ __forceinline__ void apply_bucket(uint4 (&acc)[T], const uint4 v, const uint32_t (&qw)[T],
                                             const int bit)
{
#pragma unroll
    for (int r = 0; r < T; ++r) {
        if constexpr (KIND == KIND_MASK) {
            const uint32_t m = 0u - ((qw[r] >> bit) & 1u);
            acc[r].x = xor_and(acc[r].x, v.x, m);
            acc[r].y = xor_and(acc[r].y, v.y, m);
            acc[r].z = xor_and(acc[r].z, v.z, m);
            acc[r].w = xor_and(acc[r].w, v.w, m);
        } else {
            if ((qw[r] >> bit) & 1u) {
                acc[r].x ^= v.x;
                acc[r].y ^= v.y;
                acc[r].z ^= v.z;
                acc[r].w ^= v.w;
            }
        }
    }
}

// Accumulate buckets [jb, je) (jb a multiple of 32) of column `colc` for the
// T request rows starting at r0 into acc. Rows >= B contribute nothing. One
// loop iteration consumes one 32-bit request word; its 32 buckets are fully
// unrolled so every bit test has a constant position (one s_bfe_i32 for the
// mask, or one s_bitcmp1 + branch for the zero-skip). Loads of D run U
// buckets ahead, across word boundaries; the database has
// padded_db_rows(n) readable rows, so whole words and the prefetch past the
// range end need no clamping (those rows only meet request bits that are
// zero). The row address is wave-uniform (SGPRs, advanced by the stride)
// and the lane adds a fixed byte offset, so each load is one
// global_load_dwordx4 with saddr + voffset.
template <int T, int KIND, int U>
__device__ __forceinline__ void tile_accumulate(uint4 (&acc)[T], const uint4 *__restrict__ D, uint32_t stride16,
                                                uint64_t n, const uint32_t *__restrict__ Q, uint64_t qpitch_w,
                                                uint32_t B, uint32_t r0, uint32_t colc, uint64_t jb, uint64_t je)
{
    static_assert(32 % U == 0, "unroll must divide 32");
#pragma unroll
    for (int r = 0; r < T; ++r)
        acc[r] = make_uint4(0u, 0u, 0u, 0u);
    if (jb >= je)
        return;
    const uint64_t row_bytes = (uint64_t)stride16 * 16u;
    const uint32_t lane_off = colc * 16u;
    const uint8_t *row = reinterpret_cast<const uint8_t *>(D) + jb * row_bytes;  // next row to load
    uint4 nxt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        nxt[u] = *reinterpret_cast<const uint4 *>(row + lane_off);
        row += row_bytes;
    }

    for (uint64_t j = jb; j < je; j += 32) {
        const uint64_t w = j >> 5;
        uint32_t valid = ~0u;
        if (((w + 1) << 5) > n)
            valid = (1u << (n & 31u)) - 1u;
        uint32_t qw[T];
#pragma unroll
        for (int r = 0; r < T; ++r)
            qw[r] = (r0 + r < B) ? (Q[(uint64_t)(r0 + r) * qpitch_w + w] & valid) : 0u;
#pragma unroll
        for (int c = 0; c < 32; c += U) {
            uint4 cur[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                cur[u] = nxt[u];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                nxt[u] = *reinterpret_cast<const uint4 *>(row + lane_off);
                row += row_bytes;
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                apply_bucket<T, KIND>(acc, cur[u], qw, c + u);
        }
    }
}

// SHARE = false: the 4 waves take 4 consecutive 1 KiB column chunks (one
// 4 KiB column group) of the same T request rows.
// SHARE = true: the 4 waves stream the same 1 KiB column chunk and take 4
// consecutive request tiles, so the chunk is fetched from L2 once and the
// other three waves hit in L1.
template <int T, int KIND, int U, bool SHARE>
__global__ __launch_bounds__(WG) void xorpir_tile_kernel(const TileArgs a)
{
    const uint32_t L = blockIdx.x;
    const uint32_t t = (L & 7u) * a.tasks_per_xcd + (L >> 3);
    if (t >= a.n_rt * a.n_cg * a.splits)
        return;
    const uint32_t rt = t % a.n_rt;
    const uint32_t rest = t / a.n_rt;
    const uint32_t cg = rest % a.n_cg;
    const uint32_t s = rest / a.n_cg;

    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave_col = SHARE ? cg * 64u : cg * COLS_PER_WG + wave * 64u;
    const uint32_t r0 = SHARE ? (rt * 4u + wave) * T : rt * T;
    if (wave_col >= a.stride16 || r0 >= a.B)
        return;  // nothing for this wave (no barriers follow)
    const uint32_t col = wave_col + lane;
    const bool col_ok = col < a.stride16;
    const uint32_t colc = col_ok ? col : wave_col;

    const uint64_t nwords = (a.n + 31) >> 5;
    const uint64_t wb = (uint64_t)s * a.words_per_split;
    const uint64_t we = std::min<uint64_t>(nwords, wb + a.words_per_split);
    const uint64_t jb = wb << 5;
    const uint64_t je = std::min<uint64_t>(a.n, we << 5);

    uint4 acc[T];
    tile_accumulate<T, KIND, U>(acc, a.D, a.stride16, a.n, a.Q, a.qpitch_w, a.B, r0, colc, jb, je);

    if (col_ok) {
        uint4 *o = a.out + (uint64_t)s * a.out_split16 + col;
#pragma unroll
        for (int r = 0; r < T; ++r)
            if (r0 + r < a.B)
                o[(uint64_t)(r0 + r) * a.out_row16] = acc[r];
    }
}

// resp[r][c] = XOR over s of partials[s][r][c]. A workgroup covers TI
// consecutive 16-byte words; its WG / TI thread groups take every
// (WG / TI)-th split from their own first one and combine their sums in LDS.
// Few words and many splits (a batch of one request split over every bucket
// range) thus still spread the partials over many threads.
template <int TI>
__global__ __launch_bounds__(WG) void xor_splits_kernel(const uint4 *__restrict__ P, uint64_t split16,
                                                        uint32_t splits, uint64_t count, uint32_t stride16,
                                                        uint4 *__restrict__ out, uint64_t out_row16)
{
    constexpr uint32_t TS = WG / TI;
    const uint32_t t = threadIdx.x;
    const uint32_t sg = t / TI;
    const uint64_t i = (uint64_t)blockIdx.x * TI + t % TI;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    if (i < count) {
#pragma unroll 8
        for (uint32_t s = sg; s < splits; s += TS) {
            const uint4 v = P[(uint64_t)s * split16 + i];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
    }
    if constexpr (TS > 1) {
        // groups [h, 2h) fold into groups [0, h); reads and writes of one
        // round touch disjoint slots
        __shared__ uint4 part[WG];
        part[t] = acc;
        __syncthreads();
#pragma unroll
        for (uint32_t h = TS / 2; h >= 1; h /= 2) {
            if (sg < h) {
                const uint4 v = part[t + h * TI];
                acc.x ^= v.x;
                acc.y ^= v.y;
                acc.z ^= v.z;
                acc.w ^= v.w;
                part[t] = acc;
            }
            __syncthreads();
        }
    }
    if (sg == 0 && i < count) {
        const uint64_t r = i / stride16, c = i % stride16;
        out[r * out_row16 + c] = acc;
    }
}

using TileFn = void (*)(const TileArgs);

template <int KIND, int U, bool SHARE>
TileFn pick_tile(uint32_t T)
{
    switch (T) {
    case 1: return SHARE ? nullptr : xorpir_tile_kernel<1, KIND, U, false>;
    case 2: return SHARE ? nullptr : xorpir_tile_kernel<2, KIND, U, false>;
    case 4: return xorpir_tile_kernel<4, KIND, U, SHARE>;
    case 8: return xorpir_tile_kernel<8, KIND, U, SHARE>;
    case 16: return xorpir_tile_kernel<16, KIND, U, SHARE>;
    case 24: return xorpir_tile_kernel<24, KIND, U, SHARE>;
    case 32: return xorpir_tile_kernel<32, KIND, U, SHARE>;
    default: return nullptr;
    }
}

template <int KIND>
TileFn pick_tile_u(uint32_t T, uint32_t U, bool share)
{
    switch (U) {
    case 4: return share ? pick_tile<KIND, 4, true>(T) : pick_tile<KIND, 4, false>(T);
    case 8: return share ? pick_tile<KIND, 8, true>(T) : pick_tile<KIND, 8, false>(T);
    case 16: return share ? nullptr : pick_tile<KIND, 16, false>(T);
    default: return nullptr;
    }
}

TileFn tile_fn(const Plan &p)
{
    const bool share = p.flags & PLAN_SHARED_COLUMN;
    if (p.kind == KIND_MASK)
        return pick_tile_u<KIND_MASK>(p.tile, p.unroll, share);
    if (p.kind == KIND_SKIP)
        return pick_tile_u<KIND_SKIP>(p.tile, p.unroll, share);
    return nullptr;
}

}  // namespace

bool tile_plan_supported(const Plan &p) { return tile_fn(p) != nullptr; }

// Words per workgroup of the split reduction: all 256 threads on distinct
// words while that gives at least 1024 workgroups (four per CU); fewer words
// per workgroup (at least 4, one 64-byte segment) and more threads per word
// for smaller answers, as long as every thread group has a split.
static uint32_t split_reduce_items(uint64_t count, uint32_t splits)
{
    uint32_t ti = WG;
    while (ti > 4 && (count + ti - 1) / ti < 1024 && 2ull * (WG / ti) <= splits)
        ti /= 2;
    return ti;
}

hipError_t launch_xor_splits(const void *partials, uint32_t splits, uint32_t B, uint64_t stride, void *out,
                             uint64_t out_pitch, hipStream_t stream, hipEvent_t done)
{
    const uint32_t stride16 = (uint32_t)(stride / 16);
    const uint64_t count = (uint64_t)B * stride16;
    if (count == 0)
        return done ? hipEventRecord(done, stream) : hipSuccess;
    const uint32_t ti = split_reduce_items(count, splits);
    void (*fn)(const uint4 *, uint64_t, uint32_t, uint64_t, uint32_t, uint4 *, uint64_t);
    switch (ti) {
    case 4: fn = xor_splits_kernel<4>; break;
    case 8: fn = xor_splits_kernel<8>; break;
    case 16: fn = xor_splits_kernel<16>; break;
    case 32: fn = xor_splits_kernel<32>; break;
    case 64: fn = xor_splits_kernel<64>; break;
    case 128: fn = xor_splits_kernel<128>; break;
    default: fn = xor_splits_kernel<WG>; break;
    }
    const uint32_t rgrid = (uint32_t)((count + ti - 1) / ti);
    hipExtLaunchKernelGGL(fn, dim3(rgrid), dim3(WG), 0, stream, nullptr, done, 0,
                          static_cast<const uint4 *>(partials), count, splits, count, stride16,
                          static_cast<uint4 *>(out), out_pitch / 16);
    return hipGetLastError();
}

hipError_t launch_tile_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                     hipEvent_t ee)
{
    TileFn fn = tile_fn(p);
    if (!fn)
        return hipErrorInvalidValue;
    TileArgs a{};
    a.D = static_cast<const uint4 *>(g.D);
    a.n = g.n;
    a.stride16 = (uint32_t)(g.stride / 16);
    a.B = g.B;
    a.Q = static_cast<const uint32_t *>(g.Q);
    a.qpitch_w = g.qpitch / 4;
    const bool share = p.flags & PLAN_SHARED_COLUMN;
    const uint32_t rows_per_wg = p.tile * (share ? 4u : 1u);
    a.n_rt = (g.B + rows_per_wg - 1) / rows_per_wg;
    a.n_cg = share ? (a.stride16 + 63) / 64 : (a.stride16 + COLS_PER_WG - 1) / COLS_PER_WG;
    a.splits = p.splits;
    const uint64_t nwords = (g.n + 31) / 32;
    a.words_per_split = (uint32_t)((nwords + p.splits - 1) / p.splits);
    if (p.splits > 1) {
        a.out = static_cast<uint4 *>(partials);
        a.out_row16 = a.stride16;
        a.out_split16 = (uint64_t)g.B * a.stride16;
    } else {
        a.out = static_cast<uint4 *>(g.out);
        a.out_row16 = g.out_pitch / 16;
        a.out_split16 = 0;
    }
    const uint64_t tasks = (uint64_t)a.n_rt * a.n_cg * a.splits;
    a.tasks_per_xcd = (uint32_t)((tasks + 7) / 8);
    const uint32_t grid = a.tasks_per_xcd * 8;
    hipExtLaunchKernelGGL(fn, dim3(grid), dim3(WG), 0, stream, eb, ee, 0, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.splits <= 1)
        return e;
    return launch_split_reduce(partials, p.splits, g, stream);
}

}  // namespace talek

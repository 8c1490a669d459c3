// Four-Russians XOR-PIR kernel for gfx950.
//
// The read is the GF(2) product R (B x n bits) . D (n buckets). The method
// of Four Russians (Arlazarov, Dinic, Kronrod, Faradzev 1970) groups the
// buckets 8 at a time: for group g the workgroup builds, once, the table
// T_g[e] = XOR of the buckets 8g + i for every bit i set in e (256 entries),
// and every request then adds T_g[byte g of its request row] with a single
// XOR. Per request and group that is one table read and one XOR instead of
// eight masked XORs; the table costs 255 XORs per group, shared by all the
// workgroup's requests. The result is the same exact XOR sum.
//
// Mapping:
//  * Each lane owns one 32-bit column of a 256-byte slice of the bucket rows.
//  * The table of a group lives in LDS as 256 entries x 64 lanes x 4 bytes
//    (64 KiB), double-buffered so that building group g + 1 overlaps the
//    lookups of group g with a single barrier per group.
//  * The NW waves of a workgroup split the table build: wave w builds the
//    entries whose high log2(NW) bits equal w, walking its low bits in Gray
//    code order so each entry costs one XOR and one ds_write_b32 with an
//    immediate offset. Each wave then looks up TW requests: the request byte
//    of the group, pre-scaled to an LDS offset by the request-staging pass,
//    is wave-uniform (scalar loads), the lane's address is one v_add_u32,
//    the entry one ds_read_b32 (conflict-free: 64 consecutive dwords) and the
//    accumulation one v_xor.
//  * Splits over bucket ranges and the XCD-aware task order are as in the
//    tiled kernels; partial answers are reduced by the same second pass.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace talek {

namespace {

constexpr int ENTRIES = 256;
constexpr int TABLE_DW = ENTRIES * 64;  // dwords per table buffer

struct M4rArgs {
    const uint32_t *D;
    uint64_t n;
    uint32_t stride_dw;
    uint32_t B;
    const uint32_t *Qs;   // staged request bytes as LDS offsets: Qs[g * Bp + r]
    uint32_t Bp;
    uint32_t *out;
    uint64_t out_row_dw;
    uint64_t out_split_dw;
    uint32_t n_rt, n_slices, splits, words_per_split, tasks_per_xcd;
};

template <int NW>
constexpr int log2_waves()
{
    return NW == 1 ? 0 : NW == 2 ? 1 : NW == 4 ? 2 : NW == 8 ? 3 : 4;
}

// Load the 8 bucket dwords of group g (rows clamped to the last valid one;
// clamped rows only ever meet request bits that are masked to zero).
__device__ __forceinline__ void load_group(uint32_t (&d)[8], const uint32_t *__restrict__ Dc, uint32_t stride_dw,
                                           uint64_t g, uint64_t last)
{
#pragma unroll
    for (int i = 0; i < 8; ++i)
        d[i] = Dc[std::min<uint64_t>(g * 8 + i, last) * stride_dw];
}

// Wave w writes entries (w << LB) | x for every x < 2^LB.
template <int NW>
__device__ __forceinline__ void build_table(uint32_t *__restrict__ tbl, const uint32_t (&d)[8], uint32_t wave,
                                            uint32_t lane)
{
    constexpr int LW = log2_waves<NW>();
    constexpr int LB = 8 - LW;
    uint32_t v = 0;
#pragma unroll
    for (int b = 0; b < LW; ++b)
        if ((wave >> b) & 1u)
            v ^= d[LB + b];
    uint32_t *w = tbl + ((wave << LB) * 64u + lane);
    w[0] = v;
#pragma unroll
    for (int k = 1; k < (1 << LB); ++k) {
        v ^= d[__builtin_ctz(k)];
        w[(k ^ (k >> 1)) * 64] = v;
    }
}

// acc[r] ^= T[request r's byte for this group] for the wave's TW requests.
// off[r] is that byte already scaled to a byte offset into the table (staged
// by launch_stage_group_offsets) and wave-uniform, so the lane address is
// one v_add_u32 (SGPR + VGPR), the entry one ds_read_b32 and the update one
// XOR.
template <int TW>
__device__ __forceinline__ void lookup(uint32_t (&acc)[TW], const uint8_t *tbl, const uint32_t *__restrict__ off)
{
#pragma unroll
    for (int r = 0; r < TW; ++r)
        acc[r] ^= *reinterpret_cast<const uint32_t *>(tbl + off[r]);
}

// One group step for group x = g + K (K = position of x in its request word,
// so the byte offset, the table buffer and the prefetch ring slot are all
// compile-time). ring[K] held group x, whose table was built in the previous
// step: it is refilled with group x + 4, so D loads run 3 steps ahead of use.
// Then the table of group x + 1 is built into the other buffer, group x is
// looked up, and the workgroup synchronises.
template <int NW, int TW, int K>
__device__ __forceinline__ void group_step(uint32_t (&acc)[TW], uint32_t (&ring)[4][8], uint32_t *lds,
                                           const uint32_t *__restrict__ Dc, uint32_t stride_dw, uint64_t x,
                                           uint64_t last, const uint32_t *__restrict__ q, uint32_t Bp,
                                           bool active, uint32_t wave, uint32_t lane)
{
    constexpr uint32_t buf = K & 1;
    // Unconditional on purpose: rows past the range are clamped (harmless
    // loads, a table nobody reads), and straight-line code lets the compiler
    // wait only for the loads issued three steps earlier.
    load_group(ring[K], Dc, stride_dw, x + 4, last);
    build_table<NW>(lds + (buf ^ 1u) * TABLE_DW, ring[(K + 1) & 3], wave, lane);
    if (active)
        lookup<TW>(acc, reinterpret_cast<const uint8_t *>(lds + buf * TABLE_DW + lane), q + K * Bp);
    __syncthreads();
}

// The 128 KiB table pair is static LDS so the compiler knows occupancy is one
// workgroup per CU and schedules the lookups for latency (many reads in
// flight) rather than for register count.
template <int NW, int TW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(1, NW / 4)))
void xorpir_m4r_kernel(const M4rArgs a)
{
    __shared__ uint32_t lds[2 * TABLE_DW];
    const uint32_t L = blockIdx.x;
    const uint32_t t = (L & 7u) * a.tasks_per_xcd + (L >> 3);
    if (t >= a.n_rt * a.n_slices * a.splits)
        return;
    const uint32_t rt = t % a.n_rt;
    const uint32_t rest = t / a.n_rt;
    const uint32_t slice = rest % a.n_slices;
    const uint32_t s = rest / a.n_slices;

    // wave index made provably uniform so request words stay in SGPRs
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t col = slice * 64u + lane;
    const bool col_ok = col < a.stride_dw;
    const uint32_t colc = col_ok ? col : slice * 64u;
    const uint32_t r0 = rt * (NW * TW) + wave * TW;
    const bool active = r0 < a.B;

    const uint64_t nwords = (a.n + 31) >> 5;
    const uint64_t wb = (uint64_t)s * a.words_per_split;
    const uint64_t we = std::min<uint64_t>(nwords, wb + a.words_per_split);
    const uint64_t gb = wb * 4, ge = (std::min<uint64_t>(a.n, we * 32) + 7) / 8;

    uint32_t acc[TW];
#pragma unroll
    for (int r = 0; r < TW; ++r)
        acc[r] = 0u;

    if (gb < ge) {
        const uint32_t *Dc = a.D + colc;
        const uint64_t last = a.n - 1;
        uint32_t ring[4][8];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            load_group(ring[k], Dc, a.stride_dw, gb + k, last);
        build_table<NW>(lds, ring[0], wave, lane);
        __syncthreads();
        const uint32_t *Qw = a.Qs + r0;
        // gb is a multiple of 4: each iteration consumes one request word
        uint64_t g = gb;
        for (; g + 4 <= ge; g += 4) {
            const uint32_t *q = Qw + g * a.Bp;
            group_step<NW, TW, 0>(acc, ring, lds, Dc, a.stride_dw, g, last, q, a.Bp, active, wave, lane);
            group_step<NW, TW, 1>(acc, ring, lds, Dc, a.stride_dw, g + 1, last, q, a.Bp, active, wave, lane);
            group_step<NW, TW, 2>(acc, ring, lds, Dc, a.stride_dw, g + 2, last, q, a.Bp, active, wave, lane);
            group_step<NW, TW, 3>(acc, ring, lds, Dc, a.stride_dw, g + 3, last, q, a.Bp, active, wave, lane);
        }
        if (g < ge) {  // last, partial request word
            const uint32_t *q = Qw + g * a.Bp;
            group_step<NW, TW, 0>(acc, ring, lds, Dc, a.stride_dw, g, last, q, a.Bp, active, wave, lane);
            if (g + 1 < ge)
                group_step<NW, TW, 1>(acc, ring, lds, Dc, a.stride_dw, g + 1, last, q, a.Bp, active, wave, lane);
            if (g + 2 < ge)
                group_step<NW, TW, 2>(acc, ring, lds, Dc, a.stride_dw, g + 2, last, q, a.Bp, active, wave, lane);
        }
    }

    if (active && col_ok) {
        uint32_t *o = a.out + (uint64_t)s * a.out_split_dw + col;
#pragma unroll
        for (int r = 0; r < TW; ++r)
            if (r0 + r < a.B)
                o[(uint64_t)(r0 + r) * a.out_row_dw] = acc[r];
    }
}

using M4rFn = void (*)(const M4rArgs);

M4rFn m4r_fn(uint32_t nw, uint32_t tw)
{
    if (nw == 4 && tw == 32) return xorpir_m4r_kernel<4, 32>;
    if (nw == 4 && tw == 64) return xorpir_m4r_kernel<4, 64>;
    if (nw == 8 && tw == 16) return xorpir_m4r_kernel<8, 16>;
    if (nw == 8 && tw == 32) return xorpir_m4r_kernel<8, 32>;
    if (nw == 8 && tw == 64) return xorpir_m4r_kernel<8, 64>;
    if (nw == 16 && tw == 16) return xorpir_m4r_kernel<16, 16>;
    if (nw == 16 && tw == 32) return xorpir_m4r_kernel<16, 32>;
    return nullptr;
}

}  // namespace

// Plan fields for this family: tile = requests per wave (TW), unroll = waves
// per workgroup (NW).
bool m4r_plan_supported(const Plan &p) { return m4r_fn(p.unroll, p.tile) != nullptr; }

static uint32_t padded_rows(uint32_t B) { return (B + 63) & ~63u; }

uint64_t m4r_staging_bytes(const ReadGeom &g)
{
    const uint64_t nwords = (g.n + 31) / 32;
    return ((nwords * 4 * padded_rows(g.B) * 4 + 255) & ~255ull);
}

uint32_t m4r_tasks(const ReadGeom &g, const Plan &p)
{
    const uint32_t stride_dw = (uint32_t)(g.stride / 4);
    const uint32_t slices = (stride_dw + 63) / 64;
    const uint32_t R = std::max<uint32_t>(1, p.tile * p.unroll);
    return ((g.B + R - 1) / R) * slices;
}

hipError_t launch_m4r_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                     hipEvent_t ee)
{
    M4rFn fn = m4r_fn(p.unroll, p.tile);
    if (!fn)
        return hipErrorInvalidValue;
    M4rArgs a{};
    a.D = static_cast<const uint32_t *>(g.D);
    a.n = g.n;
    a.stride_dw = (uint32_t)(g.stride / 4);
    a.B = g.B;
    // a1: stage the request words word-major next to the split partials
    a.Bp = padded_rows(g.B);
    uint32_t *qs = static_cast<uint32_t *>(partials);
    hipError_t e0 = launch_stage_group_offsets(g.Q, g.qpitch, g.B, g.n, qs, a.Bp, stream);
    if (e0 != hipSuccess)
        return e0;
    a.Qs = qs;
    partials = static_cast<uint8_t *>(partials) + m4r_staging_bytes(g);
    const uint32_t R = p.tile * p.unroll;
    a.n_rt = (g.B + R - 1) / R;
    a.n_slices = (a.stride_dw + 63) / 64;
    a.splits = p.splits;
    const uint64_t nwords = (g.n + 31) / 32;
    a.words_per_split = (uint32_t)((nwords + p.splits - 1) / p.splits);
    if (p.splits > 1) {
        a.out = static_cast<uint32_t *>(partials);
        a.out_row_dw = a.stride_dw;
        a.out_split_dw = (uint64_t)g.B * a.stride_dw;
    } else {
        a.out = static_cast<uint32_t *>(g.out);
        a.out_row_dw = g.out_pitch / 4;
        a.out_split_dw = 0;
    }
    const uint64_t tasks = (uint64_t)a.n_rt * a.n_slices * a.splits;
    a.tasks_per_xcd = (uint32_t)((tasks + 7) / 8);
    hipExtLaunchKernelGGL(fn, dim3(a.tasks_per_xcd * 8), dim3(p.unroll * 64), 0, stream, eb, ee, 0, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.splits <= 1)
        return e;
    return launch_split_reduce(partials, p.splits, g, stream);
}

}  // namespace talek

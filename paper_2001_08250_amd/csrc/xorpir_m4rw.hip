// Four-Russians XOR-PIR kernel with 16-byte table entries per lane (gfx950).
//
// Same method as xorpir_m4r.hip (Arlazarov, Dinic, Kronrod, Faradzev 1970):
// buckets are taken 6 at a time, the workgroup builds the 64 XOR
// combinations of a group once, and every request adds the combination its 6
// request bits select. Here each lane owns 16 bytes of the bucket row, so a
// table entry is a 1 KiB row slice and a lookup is one ds_read_b128: on
// gfx950 128-bit LDS reads deliver about twice the bytes per clock of 32-bit
// reads, and LDS bandwidth is what bounds this kernel. A group table is
// 64 entries x 1 KiB = 64 KiB; two of them (double buffering: build group
// x + 1 while looking up group x, one barrier per group) fill 128 KiB of LDS.
//
// Per request and group of 6 buckets: one v_add_u32 (LDS address from a
// pre-scaled, wave-uniform offset), one ds_read_b128 and four v_xor_b32 for
// 24 (bucket, dword) terms. The table costs 63 x 4 XORs and 64 ds_write_b128
// per group, split over the workgroup's waves and shared by all its requests.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace talek {

namespace {

constexpr int GB = 6;                        // buckets per group
constexpr int ENTRIES = 1 << GB;             // 64
constexpr int ENTRY_BYTES = 64 * 16;         // one 1 KiB row slice
constexpr int TABLE_U4 = ENTRIES * 64;       // uint4 per table buffer

struct WideArgs {
    const uint8_t *D;
    uint64_t row_bytes;     // stride
    uint32_t slices;        // 1 KiB column slices per row
    uint32_t stride16;
    uint32_t B;
    uint32_t Bp;            // staged rows per group (multiple of 64)
    const uint32_t *Qs;     // Qs[g * Bp + r] = (6 request bits of group g) * ENTRY_BYTES
    uint32_t *out;          // uint4 rows via out_row16 / out_split16
    uint64_t out_row16;
    uint64_t out_split16;
    uint64_t groups;        // ceil(n / 6)
    uint32_t n_rt, splits, groups_per_split, tasks_per_xcd;
    // pair-table kernel: products of `leaves` databases of one shape in one
    // launch, leaf l's at D + l * leaf_d_bytes, offsets at Qs + l * leaf_qs,
    // answers l * leaf_out16 uint4 into each split's (or the final) rows
    uint32_t leaves, tasks;
    uint64_t leaf_d_bytes, leaf_qs, leaf_out16;
};

template <int NW>
constexpr int log2_waves()
{
    return NW == 1 ? 0 : NW == 2 ? 1 : NW == 4 ? 2 : NW == 8 ? 3 : 4;
}

// The 6 bucket row slices of group g for this lane (the database has
// padded_db_rows(n) readable rows; rows past n only meet zero request bits).
__device__ __forceinline__ void load_group(uint4 (&d)[GB], const uint8_t *__restrict__ D, uint64_t row_bytes,
                                           uint32_t lane_off, uint64_t g)
{
    const uint8_t *row = D + g * GB * row_bytes;
#pragma unroll
    for (int i = 0; i < GB; ++i) {
        d[i] = *reinterpret_cast<const uint4 *>(row + lane_off);
        row += row_bytes;
    }
}

__device__ __forceinline__ void xor4(uint4 &a, const uint4 &b)
{
    a.x ^= b.x;
    a.y ^= b.y;
    a.z ^= b.z;
    a.w ^= b.w;
}

// Wave w writes entries (w << LB) | x, x < 2^LB, walking x in Gray code
// order: one 4-dword XOR and one ds_write_b128 per entry.
template <int NW>
__device__ __forceinline__ void build_table(uint4 *__restrict__ tbl, const uint4 (&d)[GB], uint32_t wave,
                                            uint32_t lane)
{
    constexpr int LW = log2_waves<NW>();
    constexpr int LB = GB - LW;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int b = 0; b < LW; ++b)
        if ((wave >> b) & 1u)
            xor4(v, d[LB + b]);
    uint4 *w = tbl + ((wave << LB) * 64u + lane);
    w[0] = v;
#pragma unroll
    for (int k = 1; k < (1 << LB); ++k) {
        xor4(v, d[__builtin_ctz(k)]);
        w[(k ^ (k >> 1)) * 64] = v;
    }
}

// Lookups in batches: BATCH ds_read_b128 in flight per wave before the first
// XOR, to cover the LDS latency (4 for 16-wave workgroups, whose waves are
// limited to 128 VGPRs, else 8).
template <int TW, int BATCH>
__device__ __forceinline__ void lookup(uint4 (&acc)[TW], const uint8_t *tbl, const uint32_t *__restrict__ off)
{
#pragma unroll
    for (int r0 = 0; r0 < TW; r0 += BATCH) {
        uint4 t[BATCH];
#pragma unroll
        for (int i = 0; i < BATCH; ++i)
            t[i] = *reinterpret_cast<const uint4 *>(tbl + off[r0 + i]);
#pragma unroll
        for (int i = 0; i < BATCH; ++i)
            xor4(acc[r0 + i], t[i]);
    }
}

// Rolling lookups: INFL ds_read_b128 stay in flight; the buffer of request r
// is refilled with request r + INFL right after its XOR, so LDS latency
// overlaps the XORs of the requests before it.
template <int TW, int INFL>
__device__ __forceinline__ void lookup_rolling(uint4 (&acc)[TW], const uint8_t *tbl, const uint32_t (&off)[TW])
{
    uint4 t[INFL];
#pragma unroll
    for (int i = 0; i < INFL; ++i)
        t[i] = *reinterpret_cast<const uint4 *>(tbl + off[i]);
#pragma unroll
    for (int r = 0; r < TW; ++r) {
        // keep this order: the scheduler would otherwise cluster the reads
        // back into batches
        __builtin_amdgcn_sched_barrier(0);
        xor4(acc[r], t[r % INFL]);
        if (r + INFL < TW)
            t[r % INFL] = *reinterpret_cast<const uint4 *>(tbl + off[r + INFL]);
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Group step for group x, K = (x - first group) mod U with U = lcm(P, 2):
// ring[K % P] held group x (already built) and is refilled with group x + P,
// so D loads run P - 1 steps ahead of their use; then group x + 1 (in
// ring[(K + 1) % P]) is built into the other table buffer, group x is looked
// up from buffer K & 1, and the workgroup synchronises. Loads and builds past
// the range are harmless (readable padding rows, a table nobody reads) and
// keep the code straight-line so the waits stay exact.
//
// MODE 0: the group's TW offsets are read (scalar loads) at its lookup and
// looked up in batches. MODE 1: offs already holds them (loaded at the end of
// the previous step, so they landed in the wait that precedes the barrier);
// lookups are rolling, and the next group's offsets are loaded after them
// (the staging area has one zero group past the end).
template <int NW, int TW, int P, int MODE, int K>
__device__ __forceinline__ void group_step(uint4 (&acc)[TW], uint4 (&ring)[P][GB], uint32_t (&offs)[TW],
                                           uint4 *lds, const uint8_t *__restrict__ D, uint64_t row_bytes,
                                           uint32_t lane_off, uint64_t x, const uint32_t *__restrict__ Qw,
                                           uint32_t Bp, bool active, uint32_t wave, uint32_t lane)
{
    constexpr int slot = K % P, next = (K + 1) % P, buf = K & 1;
    const uint32_t *q = Qw + x * Bp;
    load_group(ring[slot], D, row_bytes, lane_off, x + P);
    build_table<NW>(lds + (buf ^ 1) * TABLE_U4, ring[next], wave, lane);
    const uint8_t *tbl = reinterpret_cast<const uint8_t *>(lds + buf * TABLE_U4 + lane);
    if (active) {
        if constexpr (MODE == 1)
            lookup_rolling<TW, (NW >= 16 ? 4 : 8)>(acc, tbl, offs);
        else
            lookup<TW, (NW >= 16 ? 4 : 8)>(acc, tbl, q);
    }
    if (MODE == 1 && active) {
        // Rows r0 .. r0 + TW - 1 < Bp (r0 < B, TW divides 64) of group
        // x + 1 <= groups: inside the staging area. The group index goes
        // through readfirstlane so loop strength reduction cannot split the
        // TW addresses into separate induction pointers; they stay one base
        // plus constant offsets (wide scalar loads).
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(x + 1));
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((x + 1) >> 32));
        const uint32_t *qn = Qw + (((uint64_t)hi << 32) | lo) * Bp;
#pragma unroll
        for (int i = 0; i < TW; ++i)
            offs[i] = qn[i];
    }
    __syncthreads();
}

template <int NW, int TW, int P, int MODE, int K, int U>
__device__ __forceinline__ void group_steps(uint4 (&acc)[TW], uint4 (&ring)[P][GB], uint32_t (&offs)[TW],
                                            uint4 *lds, const uint8_t *__restrict__ D, uint64_t row_bytes,
                                            uint32_t lane_off, uint64_t x, const uint32_t *__restrict__ Qw,
                                            uint32_t Bp, bool active, uint32_t wave, uint32_t lane)
{
    if constexpr (K < U) {
        group_step<NW, TW, P, MODE, K>(acc, ring, offs, lds, D, row_bytes, lane_off, x + K, Qw, Bp,
                                       active, wave, lane);
        group_steps<NW, TW, P, MODE, K + 1, U>(acc, ring, offs, lds, D, row_bytes, lane_off, x, Qw, Bp, active,
                                               wave, lane);
    }
}

// Tail: the first `left` (< U) steps of an unrolled iteration.
template <int NW, int TW, int P, int MODE, int K, int U>
__device__ __forceinline__ void group_steps_tail(uint4 (&acc)[TW], uint4 (&ring)[P][GB], uint32_t (&offs)[TW],
                                                 uint4 *lds, const uint8_t *__restrict__ D, uint64_t row_bytes,
                                                 uint32_t lane_off, uint64_t x, uint64_t left,
                                                 const uint32_t *__restrict__ Qw, uint32_t Bp, bool active,
                                                 uint32_t wave, uint32_t lane)
{
    if constexpr (K < U) {
        if ((uint64_t)K < left) {
            group_step<NW, TW, P, MODE, K>(acc, ring, offs, lds, D, row_bytes, lane_off, x + K, Qw, Bp,
                                           active, wave, lane);
            group_steps_tail<NW, TW, P, MODE, K + 1, U>(acc, ring, offs, lds, D, row_bytes, lane_off, x, left, Qw,
                                                        Bp, active, wave, lane);
        }
    }
}

// One workgroup per CU (its two tables fill the LDS): NW / 4 waves per SIMD.
template <int NW, int TW, int P, int MODE>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
void xorpir_m4rw_kernel(const WideArgs a)
{
    constexpr int U = (P % 2 == 0) ? P : 2 * P;  // lcm(P, 2)
    __shared__ uint4 lds[2 * TABLE_U4];
    const uint32_t L = blockIdx.x;
    const uint32_t t = (L & 7u) * a.tasks_per_xcd + (L >> 3);
    if (t >= a.tasks)
        return;
    const uint32_t rt = t % a.n_rt;
    const uint32_t rest = t / a.n_rt;
    const uint32_t slice = rest % a.slices;
    const uint32_t s = rest / a.slices;

    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t col = slice * 64u + lane;
    const bool col_ok = col < a.stride16;
    const uint32_t lane_off = (col_ok ? col : slice * 64u) * 16u;
    const uint32_t r0 = rt * (NW * TW) + wave * TW;
    const bool active = r0 < a.B;

    const uint64_t gb = (uint64_t)s * a.groups_per_split;
    const uint64_t ge = std::min<uint64_t>(a.groups, gb + a.groups_per_split);

    uint4 acc[TW];
#pragma unroll
    for (int r = 0; r < TW; ++r)
        acc[r] = make_uint4(0u, 0u, 0u, 0u);

    if (gb < ge) {
        uint4 ring[P][GB];
#pragma unroll
        for (int k = 0; k < P; ++k)
            load_group(ring[k], a.D, a.row_bytes, lane_off, gb + k);
        const uint32_t *Qw = a.Qs + r0;
        uint32_t offs[TW] = {};
        if (MODE == 1 && active) {
#pragma unroll
            for (int i = 0; i < TW; ++i)
                offs[i] = Qw[gb * a.Bp + i];
        }
        build_table<NW>(lds, ring[0], wave, lane);
        __syncthreads();
        uint64_t x = gb;
        for (; x + U <= ge; x += U)
            group_steps<NW, TW, P, MODE, 0, U>(acc, ring, offs, lds, a.D, a.row_bytes, lane_off, x, Qw, a.Bp,
                                               active, wave, lane);
        if (x < ge)
            group_steps_tail<NW, TW, P, MODE, 0, U>(acc, ring, offs, lds, a.D, a.row_bytes, lane_off, x, ge - x,
                                                    Qw, a.Bp, active, wave, lane);
    }

    if (active && col_ok) {
        uint4 *o = reinterpret_cast<uint4 *>(a.out) + (uint64_t)s * a.out_split16 + col;
#pragma unroll
        for (int r = 0; r < TW; ++r)
            if (r0 + r < a.B)
                o[(uint64_t)(r0 + r) * a.out_row16] = acc[r];
    }
}

// ---- Paired G-bucket tables -------------------------------------------
//
// A step covers 2G buckets ("pair" y: buckets 2Gy .. 2Gy+2G-1) as two
// G-bucket tables A (the first G) and B (the next G) of 2^G x 1 KiB entries
// each. Every request looks up both tables and folds the two entries into its
// accumulator with one 3-input XOR per dword. Half of the waves load and build
// table A, the other half table B, so each wave holds only G row slices per
// pair in flight. Two sets of two tables (double buffering) take 2^(G+2) KiB
// of LDS: 128 KiB at G = 5 (large batches, one workgroup per CU), 64 / 32
// KiB at G = 4 / 3 (batches of tens of requests, where smaller tables cost
// fewer LDS writes per request and two workgroups share a CU). Per request
// and pair: 2 address adds, 2 ds_read_b128 and 4 v_xor3 for 2G x 4 units;
// one barrier per 2G buckets.
template <int G>
struct PairShape {
    static constexpr int E = 1 << G;             // entries per table
    static constexpr int TABLE_U4 = E * 64;      // E x 1 KiB
    static constexpr int SET_U4 = 2 * TABLE_U4;  // the two tables of a step
    static constexpr int BUCKETS = 2 * G;        // buckets per step
    static constexpr int WGS = G == 5 ? 1 : 2;   // workgroups per CU
};

// The G row slices of one half (0 = A, 1 = B) of pair y for this lane
// (rows past n are readable padding and only meet zero request bits).
template <int G>
__device__ __forceinline__ void load_half(uint4 (&d)[G], const uint8_t *__restrict__ D, uint64_t row_bytes,
                                          uint32_t lane_off, uint64_t y, uint32_t half)
{
    const uint8_t *row = D + (y * (2 * G) + half * G) * row_bytes;
#pragma unroll
    for (int i = 0; i < G; ++i) {
        d[i] = *reinterpret_cast<const uint4 *>(row + lane_off);
        row += row_bytes;
    }
}

// Wave wt of the WPT waves that build one table writes entries (wt << LB) | x,
// x < 2^LB, in Gray code order.
template <int WPT, int G>
__device__ __forceinline__ void build_half(uint4 *__restrict__ tbl, const uint4 (&d)[G], uint32_t wt, uint32_t lane)
{
    constexpr int LW = log2_waves<WPT>();
    constexpr int LB = G - LW;
    static_assert(LB >= 0, "more building waves than table entries");
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int b = 0; b < LW; ++b)
        if ((wt >> b) & 1u)
            xor4(v, d[LB + b]);
    uint4 *w = tbl + ((wt << LB) * 64u + lane);
    w[0] = v;
#pragma unroll
    for (int k = 1; k < (1 << LB); ++k) {
        xor4(v, d[__builtin_ctz(k)]);
        w[(k ^ (k >> 1)) * 64] = v;
    }
}

// a ^= b ^ c, one v_bitop3_b32 per dword (truth table 0x96 = x ^ y ^ z); the
// compiler does not fuse the two XORs by itself here.
__device__ __forceinline__ uint32_t xor3(uint32_t x, uint32_t y, uint32_t z)
{
    return __builtin_amdgcn_bitop3_b32(x, y, z, 0x96);
}

__device__ __forceinline__ void xor3x4(uint4 &a, const uint4 &b, const uint4 &c)
{
    a.x = xor3(a.x, b.x, c.x);
    a.y = xor3(a.y, b.y, c.y);
    a.z = xor3(a.z, b.z, c.z);
    a.w = xor3(a.w, b.w, c.w);
}

// Rolling pair lookups. Two forms of the staged request bits:
// H = false: off[r] holds table A's byte offset in its low half and table
// B's (set-relative, so including table A's 2^G KiB) in its high half.
// H = true: off[r / 2] holds the 2G request bits of rows r (even r in its low
// half, odd r in its high half; table A's G bits lowest); an entry is
// ENTRY_BYTES = 2^10 bytes, so each offset is one shift and one AND of the
// word (a scalar op more per offset than the first form, for half the
// staged bytes).
template <int G, int TW, bool H>
__device__ __forceinline__ uint32_t pair_off_a(const uint32_t (&off)[H ? TW / 2 : TW], int r)
{
    if constexpr (H) {
        constexpr uint32_t M = (uint32_t)((1 << G) - 1) * ENTRY_BYTES;
        const uint32_t w = off[r >> 1];
        return (r & 1) ? (w >> 6) & M : (w << 10) & M;
    } else {
        return off[r] & 0xffffu;
    }
}

template <int G, int TW, bool H>
__device__ __forceinline__ uint32_t pair_off_b(const uint32_t (&off)[H ? TW / 2 : TW], int r)
{
    if constexpr (H) {
        constexpr uint32_t M = (uint32_t)((1 << G) - 1) * ENTRY_BYTES;
        constexpr uint32_t TB = (uint32_t)(1 << G) * ENTRY_BYTES;  // table B follows table A in the set
        const uint32_t w = off[r >> 1];
        return TB + ((r & 1) ? (w >> (6 + G)) & M : (w << (10 - G)) & M);
    } else {
        return off[r] >> 16;
    }
}

template <int G, int TW, int INFL, bool H>
__device__ __forceinline__ void lookup_pairs(uint4 (&acc)[TW], const uint8_t *set,
                                             const uint32_t (&off)[H ? TW / 2 : TW])
{
    static_assert(ENTRY_BYTES == 1 << 10 && G <= 5 && TW % 2 == 0, "offsets below 64 KiB");
    uint4 ta[INFL], tb[INFL];
#pragma unroll
    for (int i = 0; i < INFL; ++i) {
        ta[i] = *reinterpret_cast<const uint4 *>(set + pair_off_a<G, TW, H>(off, i));
        tb[i] = *reinterpret_cast<const uint4 *>(set + pair_off_b<G, TW, H>(off, i));
    }
#pragma unroll
    for (int r = 0; r < TW; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        xor3x4(acc[r], ta[r % INFL], tb[r % INFL]);
        if (r + INFL < TW) {
            ta[r % INFL] = *reinterpret_cast<const uint4 *>(set + pair_off_a<G, TW, H>(off, r + INFL));
            tb[r % INFL] = *reinterpret_cast<const uint4 *>(set + pair_off_b<G, TW, H>(off, r + INFL));
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// Pair step for pair y, K = (y - first pair) mod U: ring[K % P] held this
// wave's half of pair y (already built) and is refilled with pair y + P;
// pair y is looked up; the next pair's offsets are fetched; the half of pair
// y + 1 in ring[(K + 1) % P] is built into the other set (before the lookups
// for the shapes named below); barrier.
template <int NW, int TW, int P, int K, int G, bool H>
__device__ __forceinline__ void pair_step(uint4 (&acc)[TW], uint4 (&ring)[P][G],
                                          uint32_t (&offs)[H ? TW / 2 : TW],
                                          uint4 *lds, const uint8_t *__restrict__ D, uint64_t row_bytes,
                                          uint32_t lane_off, uint64_t y, const uint32_t *__restrict__ Qw,
                                          uint32_t Bw, bool active, uint32_t half, uint32_t wt, uint32_t lane)
{
    using S = PairShape<G>;
    constexpr int slot = K % P, next = (K + 1) % P, buf = K & 1;
    // The next table is built after this step's lookups: issued first, its
    // LDS writes hold up every wave's reads (and so its XORs) at the start of
    // the step. Where two workgroups share a CU (128 VGPRs each), the longer
    // live ranges of that order fit with 2 pairs of prefetch (and, at 16
    // requests per wave, 2 lookup pairs in flight instead of 4); deeper
    // prefetch builds first.
    constexpr bool late_build = G == 5 || P <= 2;
    constexpr int in_flight = (G < 5 && TW >= 16) ? 2 : 4;
    load_half<G>(ring[slot], D, row_bytes, lane_off, y + P, half);
    if (!late_build)
        build_half<NW / 2, G>(lds + (buf ^ 1) * S::SET_U4 + half * S::TABLE_U4, ring[next], wt, lane);
    if (active) {
        lookup_pairs<G, TW, in_flight, H>(acc, reinterpret_cast<const uint8_t *>(lds + buf * S::SET_U4 + lane),
                                          offs);
        // the next pair's staged words (rows r0 .. r0 + TW - 1 < Bp of pair
        // y + 1 <= pairs, Bw words a pair, inside the staging area); the
        // index goes through readfirstlane for the reason given in group_step
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(y + 1));
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((y + 1) >> 32));
        const uint32_t *qn = Qw + (((uint64_t)hi << 32) | lo) * Bw;
#pragma unroll
        for (int i = 0; i < (H ? TW / 2 : TW); ++i)
            offs[i] = qn[i];
    }
    if (late_build)
        build_half<NW / 2, G>(lds + (buf ^ 1) * S::SET_U4 + half * S::TABLE_U4, ring[next], wt, lane);
    __syncthreads();
}

template <int NW, int TW, int P, int K, int U, int G, bool H>
__device__ __forceinline__ void pair_steps(uint4 (&acc)[TW], uint4 (&ring)[P][G],
                                           uint32_t (&offs)[H ? TW / 2 : TW], uint4 *lds,
                                           const uint8_t *__restrict__ D, uint64_t row_bytes, uint32_t lane_off,
                                           uint64_t y, const uint32_t *__restrict__ Qw, uint32_t Bp, bool active,
                                           uint32_t half, uint32_t wt, uint32_t lane)
{
    if constexpr (K < U) {
        pair_step<NW, TW, P, K, G, H>(acc, ring, offs, lds, D, row_bytes, lane_off, y + K, Qw, Bp, active, half,
                                      wt, lane);
        pair_steps<NW, TW, P, K + 1, U, G, H>(acc, ring, offs, lds, D, row_bytes, lane_off, y, Qw, Bp, active, half,
                                              wt, lane);
    }
}

template <int NW, int TW, int P, int K, int U, int G, bool H>
__device__ __forceinline__ void pair_steps_tail(uint4 (&acc)[TW], uint4 (&ring)[P][G],
                                                uint32_t (&offs)[H ? TW / 2 : TW],
                                                uint4 *lds, const uint8_t *__restrict__ D, uint64_t row_bytes,
                                                uint32_t lane_off, uint64_t y, uint64_t left,
                                                const uint32_t *__restrict__ Qw, uint32_t Bp, bool active,
                                                uint32_t half, uint32_t wt, uint32_t lane)
{
    if constexpr (K < U) {
        if ((uint64_t)K < left) {
            pair_step<NW, TW, P, K, G, H>(acc, ring, offs, lds, D, row_bytes, lane_off, y + K, Qw, Bp, active,
                                          half, wt, lane);
            pair_steps_tail<NW, TW, P, K + 1, U, G, H>(acc, ring, offs, lds, D, row_bytes, lane_off, y, left, Qw,
                                                       Bp, active, half, wt, lane);
        }
    }
}

// Same task layout and outputs as xorpir_m4rw_kernel; a.groups counts pairs.
// H: the staged request bits are 16-bit entries (launch_stage_leaf_pairs),
// else 32-bit offset pairs (stage_pair_offsets_kernel).
template <int NW, int TW, int P, int G, bool H>
__global__ __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(NW / 4 * PairShape<G>::WGS, NW / 4 * PairShape<G>::WGS)))
void xorpir_m4rp_kernel(const WideArgs a)
{
    static_assert(NW >= 4 && NW <= 16, "two tables built by NW / 2 waves each");
    using S = PairShape<G>;
    constexpr int U = (P % 2 == 0) ? P : 2 * P;
    __shared__ uint4 lds[2 * S::SET_U4];
    const uint32_t L = blockIdx.x;
    const uint32_t t = (L & 7u) * a.tasks_per_xcd + (L >> 3);
    if (t >= a.tasks)
        return;
    const uint32_t rt = t % a.n_rt;
    const uint32_t rest = t / a.n_rt;
    const uint32_t slice = rest % a.slices;
    const uint32_t rest2 = rest / a.slices;
    const uint32_t s = rest2 % a.splits;
    const uint32_t leaf = rest2 / a.splits;
    const uint8_t *D = a.D + leaf * a.leaf_d_bytes;

    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t half = wave / (NW / 2), wt = wave % (NW / 2);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t col = slice * 64u + lane;
    const bool col_ok = col < a.stride16;
    const uint32_t lane_off = (col_ok ? col : slice * 64u) * 16u;
    const uint32_t r0 = rt * (NW * TW) + wave * TW;
    const bool active = r0 < a.B;

    const uint64_t gb = (uint64_t)s * a.groups_per_split;
    const uint64_t ge = std::min<uint64_t>(a.groups, gb + a.groups_per_split);

    uint4 acc[TW];
#pragma unroll
    for (int r = 0; r < TW; ++r)
        acc[r] = make_uint4(0u, 0u, 0u, 0u);

    if (gb < ge) {
        uint4 ring[P][G];
#pragma unroll
        for (int k = 0; k < P; ++k)
            load_half<G>(ring[k], D, a.row_bytes, lane_off, gb + k, half);
        // staged words: two rows a word with 16-bit entries (r0 is even)
        constexpr int OW = H ? TW / 2 : TW;
        const uint32_t Bw = H ? a.Bp / 2 : a.Bp;
        const uint32_t *Qw = a.Qs + leaf * a.leaf_qs + (H ? r0 / 2 : r0);
        uint32_t offs[OW] = {};
        if (active) {
#pragma unroll
            for (int i = 0; i < OW; ++i)
                offs[i] = Qw[gb * Bw + i];
        }
        build_half<NW / 2, G>(lds + half * S::TABLE_U4, ring[0], wt, lane);
        __syncthreads();
        uint64_t y = gb;
        for (; y + U <= ge; y += U)
            pair_steps<NW, TW, P, 0, U, G, H>(acc, ring, offs, lds, D, a.row_bytes, lane_off, y, Qw, Bw, active,
                                           half, wt, lane);
        if (y < ge)
            pair_steps_tail<NW, TW, P, 0, U, G, H>(acc, ring, offs, lds, D, a.row_bytes, lane_off, y, ge - y, Qw,
                                                Bw, active, half, wt, lane);
    }

    if (active && col_ok) {
        uint4 *o = reinterpret_cast<uint4 *>(a.out) + leaf * a.leaf_out16 + (uint64_t)s * a.out_split16 + col;
#pragma unroll
        for (int r = 0; r < TW; ++r)
            if (r0 + r < a.B)
                o[(uint64_t)(r0 + r) * a.out_row16] = acc[r];
    }
}

// Half-wave pair tables (PLAN_HALF_WAVES): the paired tables above with
// 512-byte entries, one per 32-lane half of a wave. Each half serves its own
// request over a 512-byte column slice, so a lane holds TW / 2 accumulators
// for a wave of TW requests and a workgroup of NW waves answers NW * TW
// requests (512 at 8 x 64) from one set of tables: against the 1 KiB-entry
// form at the same registers, a table entry serves twice the requests, which
// halves the tables' LDS writes per answer byte, while the lookups move the
// same bytes. Both halves load the same D rows (one address per pair of
// lanes); each build instruction writes two entries, one per half. The
// request bits are staged as 16-bit entries (word i of a wave's pair row
// holds its requests 2i and 2i + 1), and a lane takes its request's G-bit
// index with one vector bit-field extract at its half's shift (0 or 16) and
// forms the entry address with one shift-or. G = 5: 32 KiB per set, 64 KiB
// double-buffered; G = 6: 64 / 128 KiB.
template <int G>
struct HalfShape {
    static constexpr int E = 1 << G;                 // entries per table
    static constexpr int ENTRY = 512;                // bytes per entry
    static constexpr int TABLE_U4 = E * ENTRY / 16;
    static constexpr int SET_U4 = 2 * TABLE_U4;
    static constexpr int SET_BYTES = SET_U4 * 16;
};

// Wave wt of the WPT waves that build one table: half hw of the wave writes
// entries (wt << LB) | (hw << (LB - 1)) | x, x < 2^(LB - 1), in Gray code
// order (d holds this lane's 16 bytes of the table's G rows).
template <int WPT, int G>
__device__ __forceinline__ void build_hw(uint4 *__restrict__ tbl, const uint4 (&d)[G], uint32_t wt, uint32_t lane)
{
    constexpr int LW = log2_waves<WPT>();
    constexpr int LB = G - LW;
    static_assert(LB >= 1, "each half-wave builds at least one entry");
    const uint32_t hw = lane >> 5;
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
    for (int b = 0; b < LW; ++b)
        if ((wt >> b) & 1u)
            xor4(v, d[LB + b]);
    const uint32_t m = 0u - hw;  // all ones in the upper half
    v.x ^= d[LB - 1].x & m;
    v.y ^= d[LB - 1].y & m;
    v.z ^= d[LB - 1].z & m;
    v.w ^= d[LB - 1].w & m;
    uint4 *w = tbl + (((wt << LB) | (hw << (LB - 1))) * 32u + (lane & 31u));
    w[0] = v;
#pragma unroll
    for (int k = 1; k < (1 << (LB - 1)); ++k) {
        xor4(v, d[__builtin_ctz(k)]);
        w[(k ^ (k >> 1)) * 32] = v;
    }
}

// Lookups of a wave's TW requests, two per instruction: the lane's half hs
// (0 or 16) picks its request's 16-bit entry out of off[i].
template <int G, int TWH, int INFL>
__device__ __forceinline__ void lookup_hw(uint4 (&acc)[TWH], const uint8_t *lds_bytes, uint32_t lane_base,
                                          uint32_t hs, const uint32_t (&off)[TWH])
{
    constexpr uint32_t TB = (uint32_t)HalfShape<G>::TABLE_U4 * 16;  // table B follows table A in the set
    const uint32_t hsb = hs + G;
    uint4 ta[INFL], tb[INFL];
#pragma unroll
    for (int i = 0; i < INFL; ++i) {
        ta[i] = *reinterpret_cast<const uint4 *>(lds_bytes + ((__builtin_amdgcn_ubfe(off[i], hs, G) << 9) | lane_base));
        tb[i] = *reinterpret_cast<const uint4 *>(lds_bytes + TB +
                                                 ((__builtin_amdgcn_ubfe(off[i], hsb, G) << 9) | lane_base));
    }
#pragma unroll
    for (int r = 0; r < TWH; ++r) {
        __builtin_amdgcn_sched_barrier(0);
        xor3x4(acc[r], ta[r % INFL], tb[r % INFL]);
        if (r + INFL < TWH) {
            const uint32_t w = off[r + INFL];
            ta[r % INFL] = *reinterpret_cast<const uint4 *>(lds_bytes + ((__builtin_amdgcn_ubfe(w, hs, G) << 9) | lane_base));
            tb[r % INFL] = *reinterpret_cast<const uint4 *>(lds_bytes + TB +
                                                            ((__builtin_amdgcn_ubfe(w, hsb, G) << 9) | lane_base));
        }
    }
    __builtin_amdgcn_sched_barrier(0);
}

// One pair step of the half-wave kernel (the order of pair_step).
template <int NW, int TWH, int P, int K, int G>
__device__ __forceinline__ void hw_step(uint4 (&acc)[TWH], uint4 (&ring)[P][G], uint32_t (&offs)[TWH], uint4 *lds,
                                        const uint8_t *__restrict__ D, uint64_t row_bytes, uint32_t lane_off,
                                        uint64_t y, const uint32_t *__restrict__ Qw, uint32_t Bw, bool active,
                                        uint32_t half, uint32_t wt, uint32_t lane, uint32_t hs)
{
    using S = HalfShape<G>;
    constexpr int slot = K % P, next = (K + 1) % P, buf = K & 1;
    load_half<G>(ring[slot], D, row_bytes, lane_off, y + P, half);
    if (active) {
        lookup_hw<G, TWH, 2>(acc, reinterpret_cast<const uint8_t *>(lds),
                             (uint32_t)(buf * S::SET_BYTES) | ((lane & 31u) * 16u), hs, offs);
        // the next pair's staged words (rows r0 .. r0 + 2 TWH - 1 < Bp of
        // pair y + 1 <= pairs, Bw words a pair); the index goes through
        // readfirstlane for the reason given in group_step
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(y + 1));
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((y + 1) >> 32));
        const uint32_t *qn = Qw + (((uint64_t)hi << 32) | lo) * Bw;
#pragma unroll
        for (int i = 0; i < TWH; ++i)
            offs[i] = qn[i];
    }
    build_hw<NW / 2, G>(lds + (buf ^ 1) * S::SET_U4 + half * S::TABLE_U4, ring[next], wt, lane);
    __syncthreads();
}

template <int NW, int TWH, int P, int K, int U, int G>
__device__ __forceinline__ void hw_steps(uint4 (&acc)[TWH], uint4 (&ring)[P][G], uint32_t (&offs)[TWH], uint4 *lds,
                                         const uint8_t *__restrict__ D, uint64_t row_bytes, uint32_t lane_off,
                                         uint64_t y, uint64_t left, const uint32_t *__restrict__ Qw, uint32_t Bw,
                                         bool active, uint32_t half, uint32_t wt, uint32_t lane, uint32_t hs)
{
    if constexpr (K < U) {
        if ((uint64_t)K < left) {
            hw_step<NW, TWH, P, K, G>(acc, ring, offs, lds, D, row_bytes, lane_off, y + K, Qw, Bw, active, half, wt,
                                      lane, hs);
            hw_steps<NW, TWH, P, K + 1, U, G>(acc, ring, offs, lds, D, row_bytes, lane_off, y, left, Qw, Bw, active,
                                              half, wt, lane, hs);
        }
    }
}

// Task layout and outputs of xorpir_m4rp_kernel with 512-byte column slices
// (a.slices counts them) and NW * TW requests per workgroup.
template <int NW, int TW, int P, int G>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(NW / 4, NW / 4)))
void xorpir_m4rh_kernel(const WideArgs a)
{
    static_assert(NW >= 4 && NW <= 16 && TW % 2 == 0, "two tables built by NW / 2 waves each; two requests a word");
    constexpr int TWH = TW / 2;
    using S = HalfShape<G>;
    constexpr int U = (P % 2 == 0) ? P : 2 * P;
    __shared__ uint4 lds[2 * S::SET_U4];
    const uint32_t L = blockIdx.x;
    const uint32_t t = (L & 7u) * a.tasks_per_xcd + (L >> 3);
    if (t >= a.tasks)
        return;
    const uint32_t rt = t % a.n_rt;
    const uint32_t rest = t / a.n_rt;
    const uint32_t slice = rest % a.slices;
    const uint32_t rest2 = rest / a.slices;
    const uint32_t s = rest2 % a.splits;
    const uint32_t leaf = rest2 / a.splits;
    const uint8_t *D = a.D + leaf * a.leaf_d_bytes;

    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t half = wave / (NW / 2), wt = wave % (NW / 2);
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t hw = lane >> 5, hs = hw * 16u;
    const uint32_t col = slice * 32u + (lane & 31u);
    const bool col_ok = col < a.stride16;
    const uint32_t lane_off = (col_ok ? col : slice * 32u) * 16u;
    const uint32_t r0 = rt * (NW * TW) + wave * TW;
    const bool active = r0 < a.B;

    const uint64_t gb = (uint64_t)s * a.groups_per_split;
    const uint64_t ge = std::min<uint64_t>(a.groups, gb + a.groups_per_split);

    uint4 acc[TWH];
#pragma unroll
    for (int r = 0; r < TWH; ++r)
        acc[r] = make_uint4(0u, 0u, 0u, 0u);

    if (gb < ge) {
        uint4 ring[P][G];
#pragma unroll
        for (int k = 0; k < P; ++k)
            load_half<G>(ring[k], D, a.row_bytes, lane_off, gb + k, half);
        const uint32_t Bw = a.Bp / 2;
        const uint32_t *Qw = a.Qs + leaf * a.leaf_qs + r0 / 2;
        uint32_t offs[TWH] = {};
        if (active) {
#pragma unroll
            for (int i = 0; i < TWH; ++i)
                offs[i] = Qw[gb * Bw + i];
        }
        build_hw<NW / 2, G>(lds + half * S::TABLE_U4, ring[0], wt, lane);
        __syncthreads();
        for (uint64_t y = gb; y < ge; y += U)
            hw_steps<NW, TWH, P, 0, U, G>(acc, ring, offs, lds, D, a.row_bytes, lane_off, y, ge - y, Qw, Bw, active,
                                          half, wt, lane, hs);
    }

    if (active && col_ok) {
        uint4 *o = reinterpret_cast<uint4 *>(a.out) + leaf * a.leaf_out16 + (uint64_t)s * a.out_split16 + col;
#pragma unroll
        for (int i = 0; i < TWH; ++i) {
            const uint32_t r = r0 + 2 * i + hw;
            if (r < a.B)
                o[(uint64_t)r * a.out_row16] = acc[i];
        }
    }
}

// Qs[y * Bp + r] for pair y and request row r, with a / b the G request bits
// of tables A / B (bits >= n cleared): as 32-bit entries (B << 16) | A, A =
// a * 1024 and B = b * 1024 + 2^G KiB (table B's offset within the set;
// below 64 KiB for G <= 5); as 16-bit entries a | b << G. Rows B <= r < Bp
// and the extra pair y = pairs hold zero bits. A workgroup covers 64 rows and PAIR_CHUNK pairs, whose
// 2G * PAIR_CHUNK request bits are exactly 4G words of each row: it loads
// them row by row (consecutive threads on consecutive words) into LDS, rows
// at an odd word stride, and each wave then writes a pair's 64 offsets per
// store, one row per lane.
constexpr int PAIR_CHUNK = 64;

// The staged entries of chunk steps y0 .. y0 + PAIR_CHUNK - 1 (none past
// `pairs`) of rows r0 .. r0 + 63 from their request bits in LDS (a row per
// RS-word stride, the chunk's last window padded with a zero word).
template <int G, bool H, bool NT = false>
__device__ __forceinline__ void write_pair_offsets(const uint32_t *bits, uint64_t y0, uint64_t pairs,
                                                   uint32_t *__restrict__ Qs, uint32_t Bp, uint32_t r0)
{
    using S = PairShape<G>;
    constexpr int RS = PAIR_CHUNK * S::BUCKETS / 32 + 1;
    if constexpr (H) {
        // 16-bit entries: a thread packs 8 rows of one pair into one 16-byte
        // store (r0 and Bp are multiples of 64, so every store is aligned)
        static_assert(PAIR_CHUNK * 8 % 256 == 0, "whole tasks per thread");
        for (uint32_t task = threadIdx.x; task < PAIR_CHUNK * 8; task += 256) {
            const uint32_t k = task >> 3, g8 = (task & 7u) * 8u;
            const uint64_t y = y0 + k;
            if (y > pairs)
                continue;
            const uint32_t bit = k * S::BUCKETS, j = bit >> 5, sh = bit & 31u;
            uint32_t w[4];
#pragma unroll
            for (int m = 0; m < 8; ++m) {
                const uint32_t *row = bits + (g8 + m) * RS;
                const uint64_t win = (uint64_t)row[j] | ((uint64_t)row[j + 1] << 32);
                const uint32_t v = (uint32_t)(win >> sh) & ((1u << S::BUCKETS) - 1u);
                if (m & 1)
                    w[m >> 1] |= v << 16;
                else
                    w[m >> 1] = v;
            }
            using u32x4 = __attribute__((ext_vector_type(4))) uint32_t;
            u32x4 *dst = reinterpret_cast<u32x4 *>(reinterpret_cast<uint16_t *>(Qs) + y * Bp + r0 + g8);
            const u32x4 val = {w[0], w[1], w[2], w[3]};
            if constexpr (NT)
                __builtin_nontemporal_store(val, dst);
            else
                *dst = val;
        }
        return;
    }
    const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
    for (uint32_t k = wave; k < PAIR_CHUNK; k += 4) {
        const uint64_t y = y0 + k;
        if (y > pairs)
            break;
        const uint32_t bit = k * S::BUCKETS, j = bit >> 5, sh = bit & 31u;
        const uint64_t win = (uint64_t)bits[lane * RS + j] | ((uint64_t)bits[lane * RS + j + 1] << 32);
        const uint32_t v = (uint32_t)(win >> sh) & ((1u << S::BUCKETS) - 1u);
        const uint32_t ta = (v & (S::E - 1)) * ENTRY_BYTES;
        const uint32_t tb = (v >> G) * ENTRY_BYTES + S::TABLE_U4 * 16;
        Qs[y * Bp + r0 + lane] = (tb << 16) | ta;
    }
}

template <int G, bool H>
__global__ __launch_bounds__(256) void stage_pair_offsets_kernel(const uint32_t *__restrict__ Q, uint64_t qpitch_w,
                                                                 uint32_t B, uint64_t n, uint32_t *__restrict__ Qs,
                                                                 uint32_t Bp, uint64_t pairs)
{
    using S = PairShape<G>;
    constexpr int W = PAIR_CHUNK * S::BUCKETS / 32;  // words per row and chunk (4G)
    constexpr int RS = W + 1;                        // LDS row stride, odd
    __shared__ uint32_t bits[64 * RS];
    const uint32_t t = threadIdx.x;
    const uint32_t r0 = blockIdx.y * 64;
    const uint64_t w0 = (uint64_t)blockIdx.x * W;
    const uint64_t nwords = (n + 31) >> 5;
#pragma unroll
    for (int k = 0; k < (64 * W + 255) / 256; ++k) {
        const uint32_t i = t + 256u * k;
        if (i < 64u * W) {
            const uint32_t row = i / W, w = i % W;
            const uint32_t r = r0 + row;
            const uint64_t wi = w0 + w;
            uint32_t v = 0u;
            if (r < B && wi < nwords) {
                v = Q[(uint64_t)r * qpitch_w + wi];
                if (wi == nwords - 1 && (n & 31u))
                    v &= (1u << (n & 31u)) - 1u;
            }
            bits[row * RS + w] = v;
        }
    }
    if (t < 64)
        bits[t * RS + W] = 0u;  // the high word of the chunk's last window
    __syncthreads();
    write_pair_offsets<G, H>(bits, (uint64_t)blockIdx.x * PAIR_CHUNK, pairs, Qs, Bp, r0);
}

// Pair entries (16-bit) of every leaf of a preprocessed read, staged
// straight from the request rows. Leaf l's row r is the XOR of the request
// blocks of its A-combination (lc.w[l]; block blk: row block blk >> 4, rows
// (blk >> 4) * Bq + r; column block blk & 15, bits (blk & 15) * Nq .. + Nq,
// bits >= n read as zero), and its entries are the ones
// stage_pair_offsets_kernel would stage from that row, at Qs + l * leaf_w. One launch for all leaves stands in for forming the leaf
// rows and staging every leaf in a launch of its own. blockIdx: x = 64 rows
// (the workgroups of one leaf and chunk run side by side and fill its pairs'
// offset rows together), y = leaf (the leaves that share request blocks
// follow each other), z = chunk.
// A leaf's request blocks packed in one word (so a workgroup fetches them
// with one scalar load): bits 0-3 the count, then 6 bits per block.
struct LeafCombos {
    uint32_t w[PREP_MAX_LEAVES];
};

template <int G, bool VEC>
__global__ __launch_bounds__(256) void stage_leaf_pairs_kernel(const LeafCombos lc, const uint32_t *__restrict__ Q,
                                                               uint64_t qpitch_w, uint32_t B, uint64_t n, uint32_t Bq,
                                                               uint64_t Wq, uint32_t *__restrict__ Qs, uint64_t leaf_w,
                                                               uint32_t Bp, uint64_t pairs)
{
    using S = PairShape<G>;
    constexpr int W = PAIR_CHUNK * S::BUCKETS / 32;
    constexpr int RS = W + 1;
    __shared__ uint32_t bits[64 * RS];
    const uint32_t t = threadIdx.x;
    const uint32_t leaf = blockIdx.y;
    const uint32_t r0 = blockIdx.x * 64;
    const uint64_t w0 = (uint64_t)blockIdx.z * W;
    const uint32_t lw = lc.w[leaf];
    const int cnt = lw & 15u;
    uint32_t blk[4];
#pragma unroll
    for (int e = 0; e < 4; ++e)
        blk[e] = (lw >> (4 + 6 * e)) & 63u;
    // Every thread's words of every request block are loaded before any is
    // used, so 4 x KW loads are in flight per thread: a word outside the
    // rows, the bits or the leaf's count of blocks is loaded from word 0 of
    // the requests (always present) and masked to zero. VEC: 16-byte loads
    // (the row pitch, the leaf block width Wq and W are multiples of 4
    // words, so a load never straddles a row or a block).
    constexpr int WV = VEC ? 4 : 1;                 // words per load
    constexpr int NL = 64 * W / WV;                 // loads per block and request block
    constexpr int KW = (NL + 255) / 256;
    static_assert(!VEC || W % 4 == 0, "16-byte loads cover whole chunks");
    using u32x4 = __attribute__((ext_vector_type(4))) uint32_t;
    u32x4 got[4][KW];
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const uint32_t i = t + 256u * k;
        const uint32_t row = i / (W / WV), w = (i % (W / WV)) * WV;
        const uint32_t lr = r0 + row;
        const uint64_t wi = w0 + w;
        const bool in = i < (uint32_t)NL && lr < Bq && wi < Wq;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint64_t r = (uint64_t)(blk[e] >> 4) * Bq + lr;
            const uint64_t sw = (blk[e] & 15u) * Wq + wi;
            const uint64_t bit = sw * 32;
            const bool ok = in && e < cnt && r < B && bit < n;
            const uint64_t at = ok ? r * qpitch_w + sw : 0;
            if constexpr (VEC) {
                u32x4 v = *reinterpret_cast<const u32x4 *>(Q + at);
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    const uint64_t b = bit + 32u * c;
                    v[c] &= (!ok || b >= n) ? 0u : b + 32 > n ? (1u << (n - b)) - 1u : ~0u;
                }
                got[e][k] = v;
            } else {
                const uint32_t keep = !ok ? 0u : bit + 32 > n ? (1u << (n - bit)) - 1u : ~0u;
                got[e][k][0] = Q[at] & keep;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < KW; ++k) {
        const uint32_t i = t + 256u * k;
        if (i < (uint32_t)NL) {
            const uint32_t row = i / (W / WV), w = (i % (W / WV)) * WV;
#pragma unroll
            for (int c = 0; c < WV; ++c)
                bits[row * RS + w + c] = got[0][k][c] ^ got[1][k][c] ^ got[2][k][c] ^ got[3][k][c];
        }
    }
    if (t < 64)
        bits[t * RS + W] = 0u;
    __syncthreads();
    write_pair_offsets<G, true, true>(bits, (uint64_t)blockIdx.z * PAIR_CHUNK, pairs, Qs + leaf * leaf_w, Bp, r0);
}

// Qs[g * Bp + r] = (bits 6g .. 6g+5 of request row r, bits >= n cleared) *
// ENTRY_BYTES; rows B <= r < Bp and the extra group g = groups are zero. One
// thread per (chunk of 32 groups, row): the chunk's 192 request bits are
// exactly words 6c .. 6c+5 of the row, and a wave covers 64 consecutive rows,
// so each group's 64 offsets go out as one contiguous store.
constexpr int STAGE_CHUNK = 32;  // groups per thread (32 x 6 bits = 6 words)

__global__ __launch_bounds__(256) void stage_wide_offsets_kernel(const uint32_t *__restrict__ Q, uint64_t qpitch_w,
                                                                 uint32_t B, uint64_t n, uint32_t *__restrict__ Qs,
                                                                 uint32_t Bp, uint64_t groups)
{
    const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    const uint64_t chunks = (groups + 1 + STAGE_CHUNK - 1) / STAGE_CHUNK;
    const uint64_t c = t / Bp;
    const uint32_t r = (uint32_t)(t % Bp);
    if (c >= chunks)
        return;
    const uint64_t nwords = (n + 31) >> 5;
    uint32_t w[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const uint64_t wi = c * 6 + j;
        w[j] = (j < 6 && r < B && wi < nwords) ? Q[(uint64_t)r * qpitch_w + wi] : 0u;
    }
    const uint64_t g0 = c * STAGE_CHUNK;
#pragma unroll
    for (int k = 0; k < STAGE_CHUNK; ++k) {
        const uint64_t g = g0 + k;
        if (g > groups)
            break;
        const int j = (6 * k) >> 5, sh = (6 * k) & 31;
        const uint64_t win = (uint64_t)w[j] | ((uint64_t)w[j + 1] << 32);
        uint32_t v = (uint32_t)(win >> sh) & (ENTRIES - 1);
        const uint64_t bit = g * GB;
        if (bit + GB > n)
            v &= bit >= n ? 0u : (1u << (n - bit)) - 1u;
        Qs[g * Bp + r] = v * ENTRY_BYTES;
    }
}

using WideFn = void (*)(const WideArgs);

// Prefetch depth comes from plan flags bits 8..11 (0 = 2 steps), the
// lookup mode from bit 12 (PLAN_ROLLING); bit 13 (PLAN_PAIRS) selects the
// paired 5-bucket tables (rolling lookups always).
WideFn wide_fn(uint32_t nw, uint32_t tw, uint32_t depth, uint32_t mode)
{
    if (depth == 0)
        depth = 2;
    if (mode == 0) {
        if (nw == 4 && tw == 32 && depth == 2) return xorpir_m4rw_kernel<4, 32, 2, 0>;
        if (nw == 8 && tw == 16 && depth == 2) return xorpir_m4rw_kernel<8, 16, 2, 0>;
        if (nw == 8 && tw == 16 && depth == 4) return xorpir_m4rw_kernel<8, 16, 4, 0>;
        if (nw == 8 && tw == 32 && depth == 2) return xorpir_m4rw_kernel<8, 32, 2, 0>;
        if (nw == 8 && tw == 32 && depth == 3) return xorpir_m4rw_kernel<8, 32, 3, 0>;
        if (nw == 16 && tw == 16 && depth == 2) return xorpir_m4rw_kernel<16, 16, 2, 0>;
    } else {
        if (nw == 4 && tw == 8 && depth == 2) return xorpir_m4rw_kernel<4, 8, 2, 1>;
        if (nw == 4 && tw == 16 && depth == 2) return xorpir_m4rw_kernel<4, 16, 2, 1>;
        if (nw == 8 && tw == 8 && depth == 2) return xorpir_m4rw_kernel<8, 8, 2, 1>;
        if (nw == 8 && tw == 16 && depth == 2) return xorpir_m4rw_kernel<8, 16, 2, 1>;
        if (nw == 8 && tw == 16 && depth == 3) return xorpir_m4rw_kernel<8, 16, 3, 1>;
        if (nw == 8 && tw == 32 && depth == 2) return xorpir_m4rw_kernel<8, 32, 2, 1>;
        if (nw == 16 && tw == 16 && depth == 2) return xorpir_m4rw_kernel<16, 16, 2, 1>;
    }
    return nullptr;
}

template <bool H>
WideFn pair_fn_h(uint32_t nw, uint32_t tw, uint32_t depth, uint32_t g)
{
    if (depth == 0)
        depth = 2;
    if (g == 5) {
        if (nw == 4 && tw == 16 && depth == 2) return xorpir_m4rp_kernel<4, 16, 2, 5, H>;
        if (nw == 4 && tw == 32 && depth == 2) return xorpir_m4rp_kernel<4, 32, 2, 5, H>;
        if (nw == 8 && tw == 4 && depth == 4) return xorpir_m4rp_kernel<8, 4, 4, 5, H>;
        if (nw == 8 && tw == 8 && depth == 2) return xorpir_m4rp_kernel<8, 8, 2, 5, H>;
        if (nw == 8 && tw == 8 && depth == 4) return xorpir_m4rp_kernel<8, 8, 4, 5, H>;
        if (nw == 8 && tw == 16 && depth == 2) return xorpir_m4rp_kernel<8, 16, 2, 5, H>;
        if (nw == 8 && tw == 16 && depth == 4) return xorpir_m4rp_kernel<8, 16, 4, 5, H>;
        if (nw == 8 && tw == 32 && depth == 2) return xorpir_m4rp_kernel<8, 32, 2, 5, H>;
        if (nw == 8 && tw == 32 && depth == 3) return xorpir_m4rp_kernel<8, 32, 3, 5, H>;
    } else if (g == 4) {
        if (nw == 8 && tw == 4 && depth == 2) return xorpir_m4rp_kernel<8, 4, 2, 4, H>;
        if (nw == 8 && tw == 4 && depth == 4) return xorpir_m4rp_kernel<8, 4, 4, 4, H>;
        if (nw == 8 && tw == 8 && depth == 2) return xorpir_m4rp_kernel<8, 8, 2, 4, H>;
        if (nw == 8 && tw == 8 && depth == 4) return xorpir_m4rp_kernel<8, 8, 4, 4, H>;
        if (nw == 8 && tw == 16 && depth == 2) return xorpir_m4rp_kernel<8, 16, 2, 4, H>;
    } else if (g == 3) {
        if (nw == 8 && tw == 4 && depth == 2) return xorpir_m4rp_kernel<8, 4, 2, 3, H>;
        if (nw == 8 && tw == 4 && depth == 4) return xorpir_m4rp_kernel<8, 4, 4, 3, H>;
        if (nw == 8 && tw == 8 && depth == 2) return xorpir_m4rp_kernel<8, 8, 2, 3, H>;
        if (nw == 8 && tw == 8 && depth == 4) return xorpir_m4rp_kernel<8, 8, 4, 3, H>;
    }
    return nullptr;
}

WideFn pair_fn(uint32_t nw, uint32_t tw, uint32_t depth, uint32_t g, bool half)
{
    return half ? pair_fn_h<true>(nw, tw, depth, g) : pair_fn_h<false>(nw, tw, depth, g);
}

// Half-wave kernels: tw = requests per wave (two per lane pair).
WideFn hw_fn(uint32_t nw, uint32_t tw, uint32_t depth, uint32_t g)
{
    if (depth == 0)
        depth = 2;
    if (g == 5) {
        if (nw == 8 && tw == 64 && depth == 2) return xorpir_m4rh_kernel<8, 64, 2, 5>;
        if (nw == 8 && tw == 64 && depth == 3) return xorpir_m4rh_kernel<8, 64, 3, 5>;
        if (nw == 8 && tw == 32 && depth == 2) return xorpir_m4rh_kernel<8, 32, 2, 5>;
        if (nw == 4 && tw == 64 && depth == 2) return xorpir_m4rh_kernel<4, 64, 2, 5>;
    } else if (g == 6) {
        if (nw == 8 && tw == 64 && depth == 2) return xorpir_m4rh_kernel<8, 64, 2, 6>;
        if (nw == 8 && tw == 32 && depth == 2) return xorpir_m4rh_kernel<8, 32, 2, 6>;
    }
    return nullptr;
}

uint32_t plan_depth(const Plan &p) { return (p.flags >> 8) & 15u; }
uint32_t plan_pair_g(const Plan &p)
{
    return (p.flags & PLAN_PAIR_G6) ? 6u : 5u - ((p.flags >> PLAN_PAIR_G_SHIFT) & 3u);
}
bool plan_half_waves(const Plan &p) { return (p.flags & PLAN_PAIRS) && (p.flags & PLAN_HALF_WAVES); }
uint32_t plan_mode(const Plan &p) { return (p.flags & PLAN_ROLLING) ? 1u : 0u; }
bool plan_pairs(const Plan &p) { return (p.flags & PLAN_PAIRS) != 0; }

WideFn plan_fn(const Plan &p, bool half = false)
{
    // G6 only with half waves; half waves only with paired 5- or 6-bucket tables
    if (((p.flags & PLAN_PAIR_G6) || (p.flags & PLAN_HALF_WAVES)) && !plan_half_waves(p))
        return nullptr;
    if (plan_half_waves(p))
        return ((p.flags >> PLAN_PAIR_G_SHIFT) & 3u) ? nullptr
                                                      : hw_fn(p.unroll, p.tile, plan_depth(p), plan_pair_g(p));
    return plan_pairs(p) ? pair_fn(p.unroll, p.tile, plan_depth(p), plan_pair_g(p), half)
                         : wide_fn(p.unroll, p.tile, plan_depth(p), plan_mode(p));
}

uint32_t padded_rows(uint32_t B) { return (B + 63) & ~63u; }

}  // namespace

// Plan fields for this family: tile = requests per wave (TW), unroll = waves
// per workgroup (NW).
bool m4rw_plan_supported(const Plan &p) { return plan_fn(p) != nullptr; }

// Table steps of a read: 6-bucket groups, or 10-bucket pairs.
uint64_t m4rw_steps(uint64_t n, const Plan &p)
{
    if (plan_pairs(p)) {
        const uint64_t per = 2 * plan_pair_g(p);
        return (n + per - 1) / per;
    }
    return (n + GB - 1) / GB;
}

uint64_t m4rw_staging_bytes(const ReadGeom &g, const Plan &p, bool half)
{
    // 32-bit entries, or 16 bits for the half-wave kernels and the paired
    // tables' staged leaves
    const bool h16 = plan_half_waves(p) || (half && plan_pairs(p));
    return ((m4rw_steps(g.n, p) + 1) * padded_rows(g.B) * (h16 ? 2 : 4) + 255) & ~255ull;
}

bool leaf_staging_supported(const ReadGeom &g, const Plan &p, uint32_t leaves)
{
    if (p.kind != KIND_M4RW || !plan_pairs(p) || !m4rw_plan_supported(p) || g.n % 32)
        return false;
    const uint64_t chunks = (m4rw_steps(g.n, p) + 1 + PAIR_CHUNK - 1) / PAIR_CHUNK;
    return chunks <= 65535 && leaves >= 1 && leaves <= PREP_MAX_LEAVES;
}

hipError_t launch_stage_leaf_pairs(const PrepTables &t, const void *Q, uint64_t qpitch, uint32_t B, uint64_t n,
                                   const ReadGeom &g, const Plan &p, void *staged, uint64_t leaf_bytes,
                                   hipStream_t stream)
{
    if (!leaf_staging_supported(g, p, t.leaves) || (leaf_bytes & 3) || (qpitch & 3))
        return hipErrorInvalidValue;
    const uint64_t pairs = m4rw_steps(g.n, p);
    const uint32_t chunks = (uint32_t)((pairs + 1 + PAIR_CHUNK - 1) / PAIR_CHUNK);
    const uint32_t Bp = padded_rows(g.B);
    const uint32_t G = plan_pair_g(p);
    LeafCombos lc{};
    for (uint32_t l = 0; l < t.leaves; ++l) {
        if (t.a_cnt[l] > 4)
            return hipErrorInvalidValue;
        lc.w[l] = t.a_cnt[l];
        for (uint32_t e = 0; e < t.a_cnt[l]; ++e) {
            if ((t.a[l][e] >> 4) >= t.grid || (t.a[l][e] & 15u) >= t.grid)
                return hipErrorInvalidValue;
            lc.w[l] |= (uint32_t)(((t.a[l][e] >> 4) << 4 | (t.a[l][e] & 15u)) & 63u) << (4 + 6 * e);
        }
    }
    // 16-byte loads when request rows and leaf blocks start on 16 bytes and
    // a row's words (the bytes every row guarantees readable) are whole
    // 16-byte units, so no load reaches past them
    const bool vec = (qpitch % 16) == 0 && (g.n / 32) % 4 == 0 && ((n + 31) / 32) % 4 == 0 &&
                     (reinterpret_cast<uintptr_t>(Q) & 15) == 0;
    auto k = vec ? (G == 6   ? stage_leaf_pairs_kernel<6, true>
                    : G == 5 ? stage_leaf_pairs_kernel<5, true>
                    : G == 4 ? stage_leaf_pairs_kernel<4, true>
                             : stage_leaf_pairs_kernel<3, true>)
                 : (G == 6   ? stage_leaf_pairs_kernel<6, false>
                    : G == 5 ? stage_leaf_pairs_kernel<5, false>
                    : G == 4 ? stage_leaf_pairs_kernel<4, false>
                             : stage_leaf_pairs_kernel<3, false>);
    hipLaunchKernelGGL(k, dim3(Bp / 64, t.leaves, chunks), dim3(256), 0, stream, lc, static_cast<const uint32_t *>(Q),
                       qpitch / 4, B, n, g.B, g.n / 32, static_cast<uint32_t *>(staged), leaf_bytes / 4, Bp, pairs);
    return hipGetLastError();
}

uint32_t m4rw_tasks(const ReadGeom &g, const Plan &p)
{
    const uint32_t stride16 = (uint32_t)(g.stride / 16);
    const uint32_t sw = plan_half_waves(p) ? 32 : 64;  // 16-byte columns per slice
    const uint32_t slices = (stride16 + sw - 1) / sw;
    const uint32_t R = std::max<uint32_t>(1, p.tile * p.unroll);
    return ((g.B + R - 1) / R) * slices;
}

hipError_t launch_m4rw_read(const ReadGeom &g, const Plan &p, void *partials, hipStream_t stream, hipEvent_t eb,
                     hipEvent_t ee)
{
    const bool staged = g.staged && plan_pairs(p);  // 16-bit entries staged for leaves
    const bool hwp = plan_half_waves(p);              // 16-bit entries, 512-byte slices
    WideFn fn = plan_fn(p, staged);
    if (!fn)
        return hipErrorInvalidValue;
    WideArgs a{};
    a.D = static_cast<const uint8_t *>(g.D);
    a.row_bytes = g.stride;
    a.stride16 = (uint32_t)(g.stride / 16);
    a.slices = hwp ? (a.stride16 + 31) / 32 : (a.stride16 + 63) / 64;
    a.B = g.B;
    a.Bp = padded_rows(g.B);
    a.groups = m4rw_steps(g.n, p);
    uint32_t *qs = static_cast<uint32_t *>(partials);
    if (staged) {
        qs = const_cast<uint32_t *>(g.staged);
    } else {
        if (plan_pairs(p)) {
            const uint64_t chunks = (a.groups + 1 + PAIR_CHUNK - 1) / PAIR_CHUNK;
            if (chunks * 256 > 0xffffffffull)  // a grid dimension holds fewer than 2^32 work-items
                return hipErrorInvalidValue;
            const uint32_t G = plan_pair_g(p);
            auto stage = hwp ? (G == 6 ? stage_pair_offsets_kernel<6, true> : stage_pair_offsets_kernel<5, true>)
                         : G == 5 ? stage_pair_offsets_kernel<5, false>
                         : G == 4 ? stage_pair_offsets_kernel<4, false>
                                  : stage_pair_offsets_kernel<3, false>;
            hipLaunchKernelGGL(stage, dim3((uint32_t)chunks, a.Bp / 64), dim3(256), 0, stream,
                               static_cast<const uint32_t *>(g.Q), g.qpitch / 4, g.B, g.n, qs, a.Bp, a.groups);
        } else {
            const uint64_t threads = (a.groups + 1 + STAGE_CHUNK - 1) / STAGE_CHUNK * a.Bp;
            if (threads > 0xffffffffull - 255)  // a launch holds fewer than 2^32 work-items
                return hipErrorInvalidValue;
            hipLaunchKernelGGL(stage_wide_offsets_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0,
                               stream, static_cast<const uint32_t *>(g.Q), g.qpitch / 4, g.B, g.n, qs, a.Bp,
                               a.groups);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    a.Qs = qs;
    if (!staged)
        partials = static_cast<uint8_t *>(partials) + m4rw_staging_bytes(g, p, false);
    const uint32_t R = p.tile * p.unroll;
    a.n_rt = (g.B + R - 1) / R;
    a.splits = p.splits;
    a.groups_per_split = (uint32_t)((a.groups + p.splits - 1) / p.splits);
    // leaves > 1: the leaves' answers are rows l * B + r of one [leaves * B]
    // row block, split by split, so one reduction serves them all
    a.leaves = g.leaves;
    a.leaf_d_bytes = g.leaf_d_bytes;
    a.leaf_qs = g.leaf_stage_bytes / 4;
    if (p.splits > 1) {
        a.out = static_cast<uint32_t *>(partials);
        a.out_row16 = a.stride16;
        a.leaf_out16 = (uint64_t)g.B * a.stride16;
        a.out_split16 = (uint64_t)g.leaves * g.B * a.stride16;
    } else {
        a.out = static_cast<uint32_t *>(g.out);
        a.out_row16 = g.out_pitch / 16;
        a.leaf_out16 = (uint64_t)g.B * a.out_row16;
        a.out_split16 = 0;
    }
    const uint64_t tasks = (uint64_t)a.n_rt * a.slices * a.splits * g.leaves;
    if ((tasks + 7) / 8 * 8 * p.unroll * 64 > 0xffffffffull)  // a launch holds fewer than 2^32 work-items
        return hipErrorInvalidValue;
    a.tasks = (uint32_t)tasks;
    a.tasks_per_xcd = (uint32_t)((tasks + 7) / 8);
    hipExtLaunchKernelGGL(fn, dim3(a.tasks_per_xcd * 8), dim3(p.unroll * 64), 0, stream, eb, ee, 0, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || p.splits <= 1)
        return e;
    ReadGeom all = g;
    all.B = g.leaves * g.B;
    return launch_split_reduce(partials, p.splits, all, stream);
}

}  // namespace talek

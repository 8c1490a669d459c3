// Preprocessed reads for large batches: Strassen's recursion over GF(2) on
// top of the Four-Russians kernels.
//
// The answers of a batch are the GF(2) product C = A D of the request bits
// A (B x n) and the database D (n x c bytes, one bucket per row). One level
// of Strassen's scheme splits A, D and C into 2 x 2 blocks and forms C from
// seven block products instead of eight (over GF(2) every sign is +, so
// each block sum is an XOR):
//   M1 = (A11 + A22)(D11 + D22)   -> C11, C22
//   M2 = (A21 + A22) D11          -> C21, C22
//   M3 = A11 (D12 + D22)          -> C12, C22
//   M4 = A22 (D21 + D11)          -> C11, C21
//   M5 = (A11 + A12) D22          -> C11, C12
//   M6 = (A21 + A11)(D11 + D12)   -> C22
//   M7 = (A12 + A22)(D21 + D22)   -> C11
// Applied L times this gives 7^L leaf products of (B / 2^L) x (n / 2^L)
// request blocks with (n / 2^L) x (c / 2^L) database blocks. The database
// side of every leaf (an XOR of at most 2^L blocks of D) depends only on the
// snapshot, so it is formed once per epoch commit: the preprocessing, which
// costs 7^L / 4^L times the snapshot in memory and one pass over it per
// commit, and saves 1 - 7^L / 8^L of the product's work on every large read.
// The request side (XORs of bit blocks) and the output side (each C block is
// the XOR of the leaf products that reach it) are formed per read.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace talek {

namespace {

constexpr int WG = 256;

// One Strassen product: the blocks (row * 2 + col) of A and D it sums, and
// the blocks of C it is added into.
struct Term {
    int a[2], na;
    int d[2], nd;
    int c[2], nc;
};
constexpr Term TERMS[7] = {
    {{0, 3}, 2, {0, 3}, 2, {0, 3}, 2},  // M1
    {{2, 3}, 2, {0, 0}, 1, {2, 3}, 2},  // M2
    {{0, 0}, 1, {1, 3}, 2, {1, 3}, 2},  // M3
    {{3, 0}, 1, {2, 0}, 2, {0, 2}, 2},  // M4
    {{0, 1}, 2, {3, 0}, 1, {0, 1}, 2},  // M5
    {{2, 0}, 2, {0, 1}, 2, {3, 0}, 1},  // M6
    {{1, 3}, 2, {2, 3}, 2, {0, 0}, 1},  // M7
};

struct Node {
    int na, nd, nc;
    uint8_t a[4], d[4], c[4];  // (row << 4) | col in the grid of the level
};

// Children of a node one level down (grid g -> 2g).
void expand(const Node &x, Node (&out)[7])
{
    for (int t = 0; t < 7; ++t) {
        const Term &T = TERMS[t];
        Node &y = out[t];
        y.na = y.nd = y.nc = 0;
        for (int i = 0; i < x.na; ++i)
            for (int k = 0; k < T.na; ++k) {
                const int r = x.a[i] >> 4, c = x.a[i] & 15, q = T.a[k];
                y.a[y.na++] = (uint8_t)(((2 * r + (q >> 1)) << 4) | (2 * c + (q & 1)));
            }
        for (int i = 0; i < x.nd; ++i)
            for (int k = 0; k < T.nd; ++k) {
                const int r = x.d[i] >> 4, c = x.d[i] & 15, q = T.d[k];
                y.d[y.nd++] = (uint8_t)(((2 * r + (q >> 1)) << 4) | (2 * c + (q & 1)));
            }
        for (int i = 0; i < x.nc; ++i)
            for (int k = 0; k < T.nc; ++k) {
                const int r = x.c[i] >> 4, c = x.c[i] & 15, q = T.c[k];
                y.c[y.nc++] = (uint8_t)(((2 * r + (q >> 1)) << 4) | (2 * c + (q & 1)));
            }
    }
}

// D-side leaf: out[row][c16] = XOR over the leaf's blocks (j, k) of
// D[j * Nq + row][k * Cq16 + c16], rows j * Nq + row >= n reading as zero.
// A workgroup takes RB = max(1, WG / Cq16) rows at a time: thread t owns
// column t mod Cq16 (and every WG-th one after it when Cq16 > WG) of row
// t / Cq16, so consecutive threads write consecutive 16-byte words. Grid:
// x = leaf, y over the rows, so the leaves that read the same rows of D run
// next to each other and share them through the caches.
__global__ __launch_bounds__(WG) void prep_d_kernel(const PrepTables t, const uint4 *__restrict__ D,
                                                    uint64_t stride16, uint64_t n, uint64_t Nq, uint32_t Cq16,
                                                    uint4 *__restrict__ out, uint64_t leaf_u4)
{
    const uint32_t leaf = blockIdx.x;
    uint4 *o = out + leaf * leaf_u4;
    const int cnt = t.d_cnt[leaf];
    const uint32_t rb = Cq16 >= WG ? 1u : WG / Cq16;
    const uint32_t rr = Cq16 >= WG ? 0u : threadIdx.x / Cq16;
    const uint32_t c0 = Cq16 >= WG ? threadIdx.x : threadIdx.x % Cq16;
    if (rr >= rb)
        return;
    for (uint64_t row = (uint64_t)blockIdx.y * rb + rr; row < Nq; row += (uint64_t)gridDim.y * rb) {
        for (uint32_t c16 = c0; c16 < Cq16; c16 += WG) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            for (int e = 0; e < cnt; ++e) {
                const uint32_t blk = t.d[leaf][e];
                const uint64_t src = (blk >> 4) * Nq + row;
                if (src < n) {
                    const uint4 x = D[src * stride16 + (blk & 15u) * Cq16 + c16];
                    v.x ^= x.x;
                    v.y ^= x.y;
                    v.z ^= x.z;
                    v.w ^= x.w;
                }
            }
            o[row * Cq16 + c16] = v;
        }
    }
}

// The same leaf rows, for the rows that buckets idx[0 .. count) feed: bucket
// b = i * Nq + x of the snapshot enters row x of a leaf through the leaf's
// blocks of row-block i only, so after a commit that changed those buckets
// the leaf rows x = b mod Nq are recomputed in full from the new snapshot
// (two changed buckets with the same x recompute the same row to the same
// bytes). Grid: x = leaf, y over the listed buckets; RB rows per workgroup as
// in prep_d_kernel.
__global__ __launch_bounds__(WG) void prep_rows_kernel(const PrepTables t, const uint4 *__restrict__ D,
                                                       uint64_t stride16, uint64_t n, uint64_t Nq, uint32_t Cq16,
                                                       const uint64_t *__restrict__ idx, uint64_t count,
                                                       uint4 *__restrict__ out, uint64_t leaf_u4)
{
    const uint32_t leaf = blockIdx.x;
    uint4 *o = out + leaf * leaf_u4;
    const int cnt = t.d_cnt[leaf];
    const uint32_t rb = Cq16 >= WG ? 1u : WG / Cq16;
    const uint32_t rr = Cq16 >= WG ? 0u : threadIdx.x / Cq16;
    const uint32_t c0 = Cq16 >= WG ? threadIdx.x : threadIdx.x % Cq16;
    if (rr >= rb)
        return;
    for (uint64_t k = (uint64_t)blockIdx.y * rb + rr; k < count; k += (uint64_t)gridDim.y * rb) {
        const uint64_t row = idx[k] % Nq;
        for (uint32_t c16 = c0; c16 < Cq16; c16 += WG) {
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            for (int e = 0; e < cnt; ++e) {
                const uint32_t blk = t.d[leaf][e];
                const uint64_t src = (blk >> 4) * Nq + row;
                if (src < n) {
                    const uint4 x = D[src * stride16 + (blk & 15u) * Cq16 + c16];
                    v.x ^= x.x;
                    v.y ^= x.y;
                    v.z ^= x.z;
                    v.w ^= x.w;
                }
            }
            o[row * Cq16 + c16] = v;
        }
    }
}

// Request-side leaf: out[row][w] = XOR over the leaf's blocks (i, j) of
// word j * Wq + w of request row i * Bq + row; rows >= B and bits >= n read
// as zero (no word wholly past bit n is read). Grid: x over the words of a
// row, y = leaf, z over the rows; a thread takes QR rows gridDim.z apart at
// a time (independent loads in flight), and the leaves that read one request
// row run next to each other.
constexpr uint32_t QR = 4;

__global__ __launch_bounds__(WG) void prep_q_kernel(const PrepTables t, const uint32_t *__restrict__ Q,
                                                    uint64_t qpitch_w, uint32_t B, uint64_t n, uint32_t Bq,
                                                    uint64_t Wq, uint32_t *__restrict__ out, uint64_t out_pitch_w,
                                                    uint64_t leaf_w)
{
    const uint32_t leaf = blockIdx.y;
    const int cnt = t.a_cnt[leaf];
    const uint32_t gz = gridDim.z;
    uint32_t *o = out + leaf * leaf_w;
    for (uint32_t row0 = blockIdx.z; row0 < Bq; row0 += gz * QR) {
        for (uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x; w < Wq; w += (uint64_t)gridDim.x * WG) {
            uint32_t v[QR] = {};
            for (int e = 0; e < cnt; ++e) {
                const uint32_t blk = t.a[leaf][e];
                const uint64_t sw = (blk & 15u) * Wq + w;
                const uint64_t bit = sw * 32;
                if (bit >= n)
                    continue;
                const uint32_t keep = bit + 32 > n ? (1u << (n - bit)) - 1u : ~0u;
#pragma unroll
                for (uint32_t k = 0; k < QR; ++k) {
                    const uint32_t row = row0 + k * gz;
                    const uint64_t r = (uint64_t)(blk >> 4) * Bq + row;
                    if (row < Bq && r < B)
                        v[k] ^= Q[r * qpitch_w + sw] & keep;
                }
            }
#pragma unroll
            for (uint32_t k = 0; k < QR; ++k) {
                const uint32_t row = row0 + k * gz;
                if (row < Bq)
                    o[(uint64_t)row * out_pitch_w + w] = v[k];
            }
        }
    }
}

// Output side, C block blockIdx.y = (bi, bk): row bi * Bq + row < B, columns
// bk * Cq16 + cc of C = XOR of the leaf products that reach the block, at
// (row, cc).
__global__ __launch_bounds__(WG) void prep_out_kernel(const PrepTables t, const uint4 *__restrict__ leaves,
                                                      uint64_t leaf_u4, uint32_t B, uint32_t Bq, uint32_t Cq16,
                                                      uint4 *__restrict__ out, uint64_t out_row16)
{
    const uint32_t blk = blockIdx.y;
    const uint32_t bi = blk / t.grid, bk = blk % t.grid;
    const uint64_t total = (uint64_t)Bq * Cq16;
    const int cnt = t.o_cnt[blk];
    for (uint64_t i = (uint64_t)blockIdx.x * WG + threadIdx.x; i < total; i += (uint64_t)gridDim.x * WG) {
        const uint32_t row = (uint32_t)(i / Cq16);
        const uint32_t r = bi * Bq + row;
        if (r >= B)
            break;  // i only grows, and with it row
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        for (int e = 0; e < cnt; ++e) {
            const uint4 x = leaves[t.o_leaf[blk][e] * leaf_u4 + i];
            v.x ^= x.x;
            v.y ^= x.y;
            v.z ^= x.z;
            v.w ^= x.w;
        }
        out[(uint64_t)r * out_row16 + (uint64_t)bk * Cq16 + i % Cq16] = v;
    }
}

uint32_t grid_for(uint64_t threads)
{
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((threads + WG - 1) / WG, 8192));
}

}  // namespace

bool prep_tables(uint32_t levels, PrepTables *t)
{
    if (levels < 1 || levels > PREP_MAX_LEVELS)
        return false;
    *t = PrepTables{};
    Node cur[PREP_MAX_LEAVES], next[PREP_MAX_LEAVES];
    cur[0] = Node{1, 1, 1, {0}, {0}, {0}};
    uint32_t count = 1;
    for (uint32_t l = 0; l < levels; ++l) {
        for (uint32_t i = 0; i < count; ++i) {
            Node kids[7];
            expand(cur[i], kids);
            for (int k = 0; k < 7; ++k)
                next[i * 7 + k] = kids[k];
        }
        count *= 7;
        std::copy(next, next + count, cur);
    }
    const uint32_t g = 1u << levels;
    t->leaves = count;
    t->grid = g;
    for (uint32_t i = 0; i < count; ++i) {
        t->a_cnt[i] = (uint8_t)cur[i].na;
        t->d_cnt[i] = (uint8_t)cur[i].nd;
        for (int e = 0; e < cur[i].na; ++e)
            t->a[i][e] = cur[i].a[e];
        for (int e = 0; e < cur[i].nd; ++e)
            t->d[i][e] = cur[i].d[e];
        for (int e = 0; e < cur[i].nc; ++e) {
            const uint32_t blk = (cur[i].c[e] >> 4) * g + (cur[i].c[e] & 15);
            t->o_leaf[blk][t->o_cnt[blk]++] = (uint8_t)i;
        }
    }
    return true;
}

hipError_t launch_prep_d(const PrepTables &t, const void *D, uint64_t stride, uint64_t n, uint64_t Nq, uint32_t Cq,
                         void *out, uint64_t leaf_bytes, hipStream_t stream)
{
    const uint32_t Cq16 = Cq / 16;
    const uint32_t rb = Cq16 >= WG ? 1u : WG / Cq16;
    const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((Nq + rb - 1) / rb, 65535));
    hipLaunchKernelGGL(prep_d_kernel, dim3(t.leaves, chunks), dim3(WG), 0, stream, t,
                       static_cast<const uint4 *>(D), stride / 16, n, Nq, Cq16, static_cast<uint4 *>(out),
                       leaf_bytes / 16);
    return hipGetLastError();
}

hipError_t launch_prep_rows(const PrepTables &t, const void *D, uint64_t stride, uint64_t n, uint64_t Nq, uint32_t Cq,
                            const uint64_t *idx, uint64_t count, void *out, uint64_t leaf_bytes, hipStream_t stream)
{
    if (count == 0)
        return hipSuccess;
    const uint32_t Cq16 = Cq / 16;
    const uint32_t rb = Cq16 >= WG ? 1u : WG / Cq16;
    const uint32_t chunks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((count + rb - 1) / rb, 65535));
    hipLaunchKernelGGL(prep_rows_kernel, dim3(t.leaves, chunks), dim3(WG), 0, stream, t,
                       static_cast<const uint4 *>(D), stride / 16, n, Nq, Cq16, idx, count,
                       static_cast<uint4 *>(out), leaf_bytes / 16);
    return hipGetLastError();
}

hipError_t launch_prep_q(const PrepTables &t, const void *Q, uint64_t qpitch, uint32_t B, uint64_t n, uint32_t Bq,
                         uint64_t Wq, void *out, uint64_t out_pitch, uint64_t leaf_bytes, hipStream_t stream)
{
    const dim3 grid(grid_for(Wq), t.leaves, std::max<uint32_t>(1, std::min<uint32_t>((Bq + QR - 1) / QR, 64)));
    hipLaunchKernelGGL(prep_q_kernel, grid, dim3(WG), 0, stream, t,
                       static_cast<const uint32_t *>(Q), qpitch / 4, B, n, Bq, Wq, static_cast<uint32_t *>(out),
                       out_pitch / 4, leaf_bytes / 4);
    return hipGetLastError();
}

hipError_t launch_prep_out(const PrepTables &t, const void *leaves, uint64_t leaf_bytes, uint32_t B, uint32_t Bq,
                           uint32_t Cq, void *out, uint64_t out_pitch, hipStream_t stream, hipEvent_t done)
{
    const uint32_t Cq16 = Cq / 16;
    hipExtLaunchKernelGGL(prep_out_kernel, dim3(grid_for((uint64_t)Bq * Cq16), t.grid * t.grid), dim3(WG), 0,
                          stream, nullptr, done, 0, t, static_cast<const uint4 *>(leaves), leaf_bytes / 16, B, Bq,
                          Cq16, static_cast<uint4 *>(out), out_pitch / 16);
    return hipGetLastError();
}

}  // namespace talek

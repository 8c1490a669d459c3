// Serialized PIR (section "Serialized PIR", steps 6 to 8): one-time masks on
// the answers and the leader's combination of the servers' masked answers.
//
// A server answers request r with R_r XOR P_r, P_r = PRNG(p_r) of the
// answer's size, p_r a per-request seed. The PRNG is ChaCha20 (32-byte key =
// the seed, 96-bit all-zero nonce, 32-bit block counter from 0): P_r is the
// first bytes of that keystream. The mask is applied where the answer is
// written: fused into the split reduction (one thread per 16-byte column and
// row, the four columns of a keystream block sharing its computation), or in
// place when the read had no bucket splits. The leader
// XORs the l servers' masked answers row by row.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "engine.h"

namespace talek {
namespace {

constexpr int WG = 256;

__device__ __forceinline__ uint32_t rotl32(uint32_t v, int c) { return __builtin_amdgcn_alignbit(v, v, 32 - c); }

__device__ __forceinline__ void qr(uint32_t &a, uint32_t &b, uint32_t &c, uint32_t &d)
{
    a += b;
    d = rotl32(d ^ a, 16);
    c += d;
    b = rotl32(b ^ c, 12);
    a += b;
    d = rotl32(d ^ a, 8);
    c += d;
    b = rotl32(b ^ c, 7);
}

// Lane i of a quad of lanes receives the value of lane (i + S) mod 4 of the
// same quad (DPP quad permutation; S is 1, 2 or 3).
template <int S>
__device__ __forceinline__ uint32_t quad_rot(uint32_t v)
{
    constexpr int ctrl = ((0 + S) & 3) | (((1 + S) & 3) << 2) | (((2 + S) & 3) << 4) | (((3 + S) & 3) << 6);
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, ctrl, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t pick4(uint32_t v0, uint32_t v1, uint32_t v2, uint32_t v3, uint32_t i)
{
    return i == 0 ? v0 : i == 1 ? v1 : i == 2 ? v2 : v3;
}

// Lane q (q = lane mod 4) of a quad holds column q of the state (words
// q, 4+q, 8+q, 12+q) in a, b, c, d: the transposed words arrive from the
// other lanes so that each lane ends with row q (words 4q .. 4q+3) in w[].
template <int S>
__device__ __forceinline__ void transpose_step(uint32_t q, uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                               uint32_t (&w)[4])
{
    // lane m sends its word of row (m - S) mod 4, the row of the lane that
    // receives it; lane q receives column (q + S) mod 4 of its own row
    const uint32_t send = pick4(a, b, c, d, (q - S) & 3u);
    const uint32_t got = S == 0 ? send : quad_rot<S & 3>(send);
    const uint32_t slot = (q + S) & 3u;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] = slot == (uint32_t)k ? got : w[k];
}

// ChaCha20 keystream block `counter` of key k (8 little-endian words, read as
// such on this little-endian device), nonce zero, computed by the four lanes
// of a quad together: lane q keeps column q of the 4 x 4 state, so a column
// round is one quarter round per lane, and a diagonal round is one quarter
// round per lane after rotating rows 1, 2, 3 of the state by 1, 2, 3 lanes
// (and back). Every lane of the quad must pass the same key and counter and
// be active. Lane q returns keystream words 4q .. 4q+3 in w[].
__device__ __forceinline__ void chacha_block_quad(const uint32_t *__restrict__ k, uint32_t counter, uint32_t q,
                                                  uint32_t (&w)[4])
{
    const uint32_t a0 = pick4(0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, q);
    const uint32_t b0 = k[q], c0 = k[4 + q], d0 = q == 0 ? counter : 0u;
    uint32_t a = a0, b = b0, c = c0, d = d0;
#pragma unroll 2
    for (int round = 0; round < 10; ++round) {
        qr(a, b, c, d);                       // columns
        b = quad_rot<1>(b);
        c = quad_rot<2>(c);
        d = quad_rot<3>(d);
        qr(a, b, c, d);                       // diagonals
        b = quad_rot<3>(b);
        c = quad_rot<2>(c);
        d = quad_rot<1>(d);
    }
    a += a0;
    b += b0;
    c += c0;
    d += d0;
    w[0] = w[1] = w[2] = w[3] = 0u;
    transpose_step<0>(q, a, b, c, d, w);
    transpose_step<1>(q, a, b, c, d, w);
    transpose_step<2>(q, a, b, c, d, w);
    transpose_step<3>(q, a, b, c, d, w);
}

// Four lanes per (row r, 64-byte keystream block j): lane q takes 16-byte
// column c = 4j + q of row r. Column c is the XOR of the splits' partials
// (or, with splits == 0, the row as it stands in out) XOR bytes 16c .. 16c+15
// of key r's keystream, i.e. words 4q .. 4q+3 of block j, which the quad
// computes once between its four lanes. Lanes of a quad whose column lies
// past the row (the row's last block) still help compute the block but
// neither read nor write. P: [splits][B][stride16].
__global__ __launch_bounds__(WG) void mask_rows_kernel(const uint4 *__restrict__ P, uint64_t split16, uint32_t splits,
                                                       uint32_t B, uint32_t stride16, uint32_t blocks_per_row,
                                                       uint4 *__restrict__ out, uint64_t out_row16,
                                                       const uint32_t *__restrict__ keys)
{
    const uint64_t t = (uint64_t)blockIdx.x * WG + threadIdx.x;
    const uint64_t quad = t >> 2;
    const uint32_t q = (uint32_t)(t & 3);
    const uint32_t r = (uint32_t)(quad / blocks_per_row), j = (uint32_t)(quad % blocks_per_row);
    if (r >= B)
        return;  // whole quads: WG and the grid are multiples of 4
    const uint32_t c = 4 * j + q;
    const bool live = c < stride16;
    uint4 *o = out + (uint64_t)r * out_row16 + c;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    if (live) {
        if (splits == 0) {
            acc = *o;
        } else {
            const uint4 *p = P + (uint64_t)r * stride16 + c;
#pragma unroll 8
            for (uint32_t s = 0; s < splits; ++s) {
                const uint4 v = p[(uint64_t)s * split16];
                acc.x ^= v.x;
                acc.y ^= v.y;
                acc.z ^= v.z;
                acc.w ^= v.w;
            }
        }
    }
    uint32_t ks[4];
    chacha_block_quad(keys + 8ull * r, j, q, ks);
    if (!live)
        return;
    acc.x ^= ks[0];
    acc.y ^= ks[1];
    acc.z ^= ks[2];
    acc.w ^= ks[3];
    *o = acc;
}

// out row r = XOR of the l input rows r.
__global__ __launch_bounds__(WG) void xor_combine_kernel(const CombineArgs a)
{
    const uint64_t t = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (uint64_t)a.B * a.row16)
        return;
    const uint64_t r = t / a.row16, c = t % a.row16;
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    for (uint32_t i = 0; i < a.l; ++i) {
        const uint4 v = a.in[i][r * a.in_row16 + c];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    a.out[r * a.out_row16 + c] = acc;
}

uint32_t blocks_for(uint64_t threads) { return (uint32_t)std::max<uint64_t>(1, (threads + WG - 1) / WG); }

}  // namespace

hipError_t launch_mask_rows(const void *partials, uint32_t splits, uint32_t B, uint64_t stride, void *out,
                            uint64_t out_pitch, const uint32_t *keys, hipStream_t stream, hipEvent_t done)
{
    if (B == 0)
        return done ? hipEventRecord(done, stream) : hipSuccess;
    const uint32_t stride16 = (uint32_t)(stride / 16);
    const uint32_t blocks_per_row = (stride16 + 3) / 4;
    const uint64_t threads = (uint64_t)B * blocks_per_row * 4;
    if (partials && splits > 1 && threads < 64ull * WG) {
        // a small answer: fewer than 64 workgroups would each walk every
        // split; the plain reduction spreads the splits over more threads,
        // then the masks go on in place
        hipError_t e = launch_xor_splits(partials, splits, B, stride, out, out_pitch, stream, nullptr);
        if (e != hipSuccess)
            return e;
        partials = nullptr;
        splits = 0;
    }
    hipExtLaunchKernelGGL(mask_rows_kernel, dim3(blocks_for(threads)), dim3(WG), 0, stream, nullptr, done, 0,
                          static_cast<const uint4 *>(partials), (uint64_t)B * stride16, splits, B, stride16,
                          blocks_per_row, static_cast<uint4 *>(out), out_pitch / 16, keys);
    return hipGetLastError();
}

hipError_t launch_xor_combine(const CombineArgs &a, hipStream_t stream)
{
    const uint64_t threads = (uint64_t)a.B * a.row16;
    if (threads == 0)
        return hipSuccess;
    hipLaunchKernelGGL(xor_combine_kernel, dim3(blocks_for(threads)), dim3(WG), 0, stream, a);
    return hipGetLastError();
}

}  // namespace talek

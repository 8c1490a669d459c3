// Serialized PIR (section "Serialized PIR", steps 6 to 8): one-time masks on
// the answers and the leader's combination of the servers' masked answers.
//
// A server answers request r with R_r XOR P_r, P_r = PRNG(p_r) of the
// answer's size, p_r a per-request seed. The PRNG is ChaCha20 (32-byte key =
// the seed, 96-bit all-zero nonce, 32-bit block counter from 0): P_r is the
// first bytes of that keystream. The mask is applied where the answer is
// written: fused into the split reduction (one thread per 16-byte column and
// row), or in place when the read had no bucket splits. The leader
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

// Keystream block `counter` of key k (8 little-endian words, read as such on
// this little-endian device), nonce zero: out[16] words.
__device__ __forceinline__ void chacha_block(const uint32_t *__restrict__ k, uint32_t counter, uint32_t (&out)[16])
{
    uint32_t x[16];
    x[0] = 0x61707865u;
    x[1] = 0x3320646eu;
    x[2] = 0x79622d32u;
    x[3] = 0x6b206574u;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        x[4 + i] = k[i];
    x[12] = counter;
    x[13] = x[14] = x[15] = 0u;
    uint32_t s[16];
#pragma unroll
    for (int i = 0; i < 16; ++i)
        s[i] = x[i];
#pragma unroll 2
    for (int round = 0; round < 10; ++round) {
        qr(x[0], x[4], x[8], x[12]);
        qr(x[1], x[5], x[9], x[13]);
        qr(x[2], x[6], x[10], x[14]);
        qr(x[3], x[7], x[11], x[15]);
        qr(x[0], x[5], x[10], x[15]);
        qr(x[1], x[6], x[11], x[12]);
        qr(x[2], x[7], x[8], x[13]);
        qr(x[3], x[4], x[9], x[14]);
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
        out[i] = x[i] + s[i];
}

// One thread per (row r, 16-byte column c): column c of row r is the XOR of
// the splits' partials (or, with splits == 0, the row as it stands in out)
// XOR bytes 16c .. 16c+15 of key r's keystream, i.e. words 4 (c mod 4) ..
// 4 (c mod 4) + 3 of block c / 4. The four threads of a block each compute
// it (a ChaCha20 block is about a thousand ALU operations), which keeps the
// split reduction as parallel as the plain one. P: [splits][B][stride16].
__global__ __launch_bounds__(WG) void mask_rows_kernel(const uint4 *__restrict__ P, uint64_t split16, uint32_t splits,
                                                       uint32_t B, uint32_t stride16, uint4 *__restrict__ out,
                                                       uint64_t out_row16, const uint32_t *__restrict__ keys)
{
    const uint64_t t = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (t >= (uint64_t)B * stride16)
        return;
    const uint32_t r = (uint32_t)(t / stride16), c = (uint32_t)(t % stride16);
    uint4 *o = out + (uint64_t)r * out_row16 + c;
    uint4 acc;
    if (splits == 0) {
        acc = *o;
    } else {
        acc = make_uint4(0u, 0u, 0u, 0u);
        const uint4 *p = P + t;
#pragma unroll 8
        for (uint32_t s = 0; s < splits; ++s) {
            const uint4 v = p[(uint64_t)s * split16];
            acc.x ^= v.x;
            acc.y ^= v.y;
            acc.z ^= v.z;
            acc.w ^= v.w;
        }
    }
    uint32_t ks[16];
    chacha_block(keys + 8ull * r, c / 4, ks);
    const uint32_t j = 4 * (c % 4);
    acc.x ^= ks[j];
    acc.y ^= ks[j + 1];
    acc.z ^= ks[j + 2];
    acc.w ^= ks[j + 3];
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
    const uint64_t threads = (uint64_t)B * stride16;
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
                          static_cast<uint4 *>(out), out_pitch / 16, keys);
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

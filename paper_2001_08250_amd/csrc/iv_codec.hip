// Compressed interest vectors (section "Private Notifications": clients fetch
// compressed Bloom-filter deltas instead of the raw vector).
//
// Stream (little-endian): m (u64), c = set bits (u64), Rice parameter
// k = floor(log2(max(1, floor(m / (c + 1))))) (u32), 4 zero bytes, then for
// the set positions in increasing order the gaps g = p - p_prev - 1 (p_prev
// starts at -1), each as floor(g / 2^k) one-bits, a zero-bit and the k low
// bits of g least significant first; bits fill bytes LSB first.
//
// Device pipeline, for a vector of W words: per-word popcounts and highest
// set bits; an exclusive sum gives every word's first code index and an
// exclusive max-scan the position set just before the word; the code lengths
// of all set bits, scanned, give their bit offsets; each set bit then ORs its
// code into the zeroed body. Only the header is assembled on the host.
#include <hip/hip_runtime.h>
#include <hipcub/device/device_scan.hpp>

#include <algorithm>
#include <vector>

#include "db.h"

namespace talek {
namespace {

constexpr int WG = 256;

__device__ __forceinline__ uint32_t valid_bits(const uint32_t *words, uint64_t w, uint64_t m)
{
    uint32_t v = words[w];
    const uint64_t lo = w * 32;
    if (lo + 32 > m)
        v &= (m > lo) ? ((1u << (m - lo)) - 1u) : 0u;
    return v;
}

__global__ __launch_bounds__(WG) void word_stats_kernel(const uint32_t *__restrict__ words, uint64_t W, uint64_t m,
                                                        uint64_t *__restrict__ counts, int64_t *__restrict__ last)
{
    const uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (w >= W)
        return;
    const uint32_t v = valid_bits(words, w, m);
    counts[w] = (uint64_t)__popc(v);
    last[w] = v ? (int64_t)(w * 32 + 31 - __clz(v)) : -1;
}

// MODE 0: code lengths into len[i]; MODE 1: codes ORed into body at off[i].
template <int MODE>
__global__ __launch_bounds__(WG) void codes_kernel(const uint32_t *__restrict__ words, uint64_t W, uint64_t m,
                                                   const uint64_t *__restrict__ base,
                                                   const int64_t *__restrict__ prev_last, uint32_t k,
                                                   uint64_t *__restrict__ len, const uint64_t *__restrict__ off,
                                                   uint32_t *__restrict__ body)
{
    const uint64_t w = (uint64_t)blockIdx.x * WG + threadIdx.x;
    if (w >= W)
        return;
    uint32_t v = valid_bits(words, w, m);
    int64_t prev = prev_last[w];
    uint64_t i = base[w];
    while (v) {
        const uint32_t b = __ffs(v) - 1;
        v &= v - 1;
        const int64_t p = (int64_t)(w * 32 + b);
        const uint64_t g = (uint64_t)(p - prev - 1);
        const uint64_t q = g >> k;
        if constexpr (MODE == 0) {
            len[i] = q + 1 + k;
        } else {
            uint64_t at = off[i];
            // q one-bits
            for (uint64_t end = at + q; at < end;) {
                const uint32_t s = (uint32_t)(at & 31);
                const uint64_t nb = std::min<uint64_t>(32 - s, end - at);
                const uint32_t mask = (nb == 32 ? 0xffffffffu : ((1u << nb) - 1u)) << s;
                atomicOr(body + (at >> 5), mask);
                at += nb;
            }
            ++at;  // the zero-bit
            // the k low bits of g, least significant first
            uint64_t r = k ? (g & ((k >= 64 ? ~0ull : (1ull << k)) - 1ull)) : 0;
            for (uint64_t end = at + k; at < end;) {
                const uint32_t s = (uint32_t)(at & 31);
                const uint64_t nb = std::min<uint64_t>(32 - s, end - at);
                const uint32_t chunk = (uint32_t)(r & (nb == 32 ? 0xffffffffull : ((1ull << nb) - 1ull)));
                if (chunk)
                    atomicOr(body + (at >> 5), chunk << s);
                r >>= nb;
                at += nb;
            }
        }
        prev = p;
        ++i;
    }
}

struct MaxOp {
    __host__ __device__ __forceinline__ int64_t operator()(int64_t a, int64_t b) const { return a > b ? a : b; }
};

uint32_t blocks(uint64_t n) { return (uint32_t)std::max<uint64_t>(1, (n + WG - 1) / WG); }

uint32_t rice_k(uint64_t m, uint64_t c)
{
    uint64_t mean = std::max<uint64_t>(1, m / (c + 1));
    uint32_t k = 0;
    while ((mean >> (k + 1)) != 0)
        ++k;
    return k;
}

}  // namespace

// Encode the m-bit device vector `words` into host memory; see the stream
// format above. out may be NULL (size query). Ordered on `s`, synchronous.
int encode_interest(pir_db *db, const uint32_t *words, uint64_t m, uint8_t *out, uint64_t cap, uint64_t *out_bytes,
                    hipStream_t s)
{
    const uint64_t W = (m + 31) / 32;
    if (W == 0 || W > 0x7fffffffull)
        return PIR_EINVAL;
    // scratch: counts, base (u64) and last, prev_last (i64), W each
    const uint64_t arr = (W * 8 + 255) & ~255ull;
    size_t t1 = 0, t2 = 0;
    if (hipcub::DeviceScan::ExclusiveSum(nullptr, t1, (uint64_t *)nullptr, (uint64_t *)nullptr, (int)W, s) !=
            hipSuccess ||
        hipcub::DeviceScan::ExclusiveScan(nullptr, t2, (int64_t *)nullptr, (int64_t *)nullptr, MaxOp(), (int64_t)-1,
                                          (int)W, s) != hipSuccess)
        return PIR_EDEVICE;
    const uint64_t tmp = (std::max<size_t>(t1, t2) + 255) & ~255ull;
    int rc = ensure_device(&db->codec, &db->codec_cap, 4 * arr + tmp);
    if (rc != PIR_OK)
        return rc;
    uint8_t *sc = static_cast<uint8_t *>(db->codec);
    uint64_t *counts = reinterpret_cast<uint64_t *>(sc);
    uint64_t *base = reinterpret_cast<uint64_t *>(sc + arr);
    int64_t *last = reinterpret_cast<int64_t *>(sc + 2 * arr);
    int64_t *prev_last = reinterpret_cast<int64_t *>(sc + 3 * arr);
    void *temp = sc + 4 * arr;
    hipLaunchKernelGGL(word_stats_kernel, dim3(blocks(W)), dim3(WG), 0, s, words, W, m, counts, last);
    if (hipGetLastError() != hipSuccess)
        return PIR_EDEVICE;
    size_t tb = tmp;
    if (hipcub::DeviceScan::ExclusiveSum(temp, tb, counts, base, (int)W, s) != hipSuccess)
        return PIR_EDEVICE;
    tb = tmp;
    if (hipcub::DeviceScan::ExclusiveScan(temp, tb, last, prev_last, MaxOp(), (int64_t)-1, (int)W, s) !=
        hipSuccess)
        return PIR_EDEVICE;
    uint64_t tail[2] = {0, 0};
    if (hipMemcpyAsync(&tail[0], base + (W - 1), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&tail[1], counts + (W - 1), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return PIR_EDEVICE;
    const uint64_t c = tail[0] + tail[1];
    if (c > 0x7fffffffull)  // the device scans count in int
        return PIR_EINVAL;
    const uint32_t k = rice_k(m, c);

    uint64_t bits = 0;
    std::vector<uint8_t> body_host;
    if (c > 0) {
        // per set bit: code length, then its bit offset
        const uint64_t carr = (c * 8 + 255) & ~255ull;
        size_t t3 = 0;
        if (hipcub::DeviceScan::ExclusiveSum(nullptr, t3, (uint64_t *)nullptr, (uint64_t *)nullptr, (int)c, s) !=
            hipSuccess)
            return PIR_EDEVICE;
        const uint64_t tmp3 = (t3 + 255) & ~255ull;
        rc = ensure_device(&db->codec2, &db->codec2_cap, 2 * carr + tmp3);
        if (rc != PIR_OK)
            return rc;
        uint8_t *sc2 = static_cast<uint8_t *>(db->codec2);
        uint64_t *len = reinterpret_cast<uint64_t *>(sc2);
        uint64_t *off = reinterpret_cast<uint64_t *>(sc2 + carr);
        hipLaunchKernelGGL(codes_kernel<0>, dim3(blocks(W)), dim3(WG), 0, s, words, W, m, base, prev_last, k, len,
                           (const uint64_t *)nullptr, (uint32_t *)nullptr);
        if (hipGetLastError() != hipSuccess)
            return PIR_EDEVICE;
        tb = tmp3;
        if (hipcub::DeviceScan::ExclusiveSum(sc2 + 2 * carr, tb, len, off, (int)c, s) != hipSuccess)
            return PIR_EDEVICE;
        uint64_t lt[2] = {0, 0};
        if (hipMemcpyAsync(&lt[0], off + (c - 1), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&lt[1], len + (c - 1), 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PIR_EDEVICE;
        bits = lt[0] + lt[1];
        const uint64_t nwords = (bits + 31) / 32;
        rc = ensure_device(&db->codec3, &db->codec3_cap, nwords * 4);
        if (rc != PIR_OK)
            return rc;
        uint32_t *body = static_cast<uint32_t *>(db->codec3);
        if (launch_fill_zero(body, nwords * 4, s) != hipSuccess)
            return PIR_EDEVICE;
        hipLaunchKernelGGL(codes_kernel<1>, dim3(blocks(W)), dim3(WG), 0, s, words, W, m, base, prev_last, k,
                           (uint64_t *)nullptr, off, body);
        if (hipGetLastError() != hipSuccess)
            return PIR_EDEVICE;
        body_host.resize((bits + 7) / 8);
        if (hipMemcpyAsync(body_host.data(), body, body_host.size(), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return PIR_EDEVICE;
    }
    const uint64_t total = 24 + (bits + 7) / 8;
    if (out_bytes)
        *out_bytes = total;
    if (!out)
        return PIR_OK;
    if (cap < total)
        return PIR_EINVAL;
    for (int i = 0; i < 8; ++i) {
        out[i] = (uint8_t)(m >> (8 * i));
        out[8 + i] = (uint8_t)(c >> (8 * i));
    }
    for (int i = 0; i < 4; ++i) {
        out[16 + i] = (uint8_t)(k >> (8 * i));
        out[20 + i] = 0;
    }
    std::copy(body_host.begin(), body_host.end(), out + 24);
    return PIR_OK;
}

}  // namespace talek

// Roofline probe for gfx950: the measured counterparts of the peaks the read
// kernels are judged against.
//   * HBM: a streaming read of a 4 GiB buffer (16 B per lane, coalesced).
//   * VALU: 32-bit bitwise operations (v_bitop3_b32, v_xor_b32) in chains
//     per lane, at several chain counts and waves per SIMD.
//   * LDS: aggregate throughput of the access patterns the Four-Russians
//     kernels use. Every lane of a wave touches consecutive bytes of one
//     contiguous row slice (64 lanes x W dwords), so the accesses are free of
//     bank conflicts; all indices stay inside the 64 KiB array. Reported per
//     CU and clock at 2.4 GHz.
//
//   ./paper_2001_08250_amd/roofline_probe
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int N = 16384;  // dwords = 64 KiB
constexpr int ITERS = 2000;

// MODE 0: reads of W dwords per lane; MODE 1: writes of W dwords per lane;
// MODE 2: four 16-byte reads per 16-byte write; MODE 3: the paired lookup of
// the Four-Russians kernels (per two 16-byte reads at wave-uniform, loop
// varying row offsets: two address adds and four three-input XORs into the
// accumulator); MODE 4: MODE 3 with two of every sixteen accesses turned into
// 16-byte writes (the lookup-to-build byte ratio of paired 32-entry tables).
template <int MODE, int W>
__global__ __launch_bounds__(256) void lds_probe(uint32_t *out, int iters)
{
    __shared__ uint32_t s[N];
    for (int i = threadIdx.x; i < N; i += 256)
        s[i] = i * 2654435761u;
    __syncthreads();
    uint4 acc = make_uint4(threadIdx.x, 1u, 2u, 3u), pa = acc;
    const int base = threadIdx.x * W;  // < 1024 dwords
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int o = base + k * 256 * W;  // <= 1020 + 15 * 1024 = 16380, +3 < N
            // row offset in [0, 15] * 1024 dwords, the same for the whole wave
            const int ov = base + (((it * 5 + k) & 15) << 10);
            if constexpr (MODE >= 3) {
                static_assert(W == 4, "paired lookups are 16 bytes per lane");
                if (MODE == 4 && k >= 14) {
                    acc.x += 1u;
                    *reinterpret_cast<uint4 *>(&s[ov]) = acc;
                } else if (k % 2 == 0) {
                    pa = *reinterpret_cast<const uint4 *>(&s[ov]);
                } else {
                    const uint4 v = *reinterpret_cast<const uint4 *>(&s[ov]);
                    acc.x = __builtin_amdgcn_bitop3_b32(acc.x, pa.x, v.x, 0x96);
                    acc.y = __builtin_amdgcn_bitop3_b32(acc.y, pa.y, v.y, 0x96);
                    acc.z = __builtin_amdgcn_bitop3_b32(acc.z, pa.z, v.z, 0x96);
                    acc.w = __builtin_amdgcn_bitop3_b32(acc.w, pa.w, v.w, 0x96);
                }
            } else if constexpr (MODE == 0) {
                if constexpr (W == 1) {
                    acc.x ^= s[o];
                } else if constexpr (W == 2) {
                    const uint2 v = *reinterpret_cast<const uint2 *>(&s[o]);
                    acc.x ^= v.x;
                    acc.y ^= v.y;
                } else {
                    const uint4 v = *reinterpret_cast<const uint4 *>(&s[o]);
                    acc.x ^= v.x;
                    acc.y ^= v.y;
                    acc.z ^= v.z;
                    acc.w ^= v.w;
                }
            } else if constexpr (MODE == 1) {
                acc.x += 1u;
                if constexpr (W == 1)
                    s[o] = acc.x;
                else if constexpr (W == 2)
                    *reinterpret_cast<uint2 *>(&s[o]) = make_uint2(acc.x, acc.y);
                else
                    *reinterpret_cast<uint4 *>(&s[o]) = acc;
            } else {
                if (k % 5 == 4) {
                    *reinterpret_cast<uint4 *>(&s[o]) = acc;
                } else {
                    const uint4 v = *reinterpret_cast<const uint4 *>(&s[o]);
                    acc.x ^= v.x;
                    acc.y ^= v.y;
                    acc.z ^= v.z;
                    acc.w ^= v.w;
                }
            }
        }
        asm volatile("" ::: "memory");  // keep every iteration's accesses
    }
    __syncthreads();
    out[blockIdx.x * 256 + threadIdx.x] = s[threadIdx.x] ^ acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// Streaming read: every element of src once, XOR-folded per thread.
__global__ __launch_bounds__(256) void hbm_read(const uint4 *__restrict__ src, uint64_t n16, uint32_t *out)
{
    uint4 acc = make_uint4(0u, 0u, 0u, 0u);
    const uint64_t stride = (uint64_t)gridDim.x * 256;
#pragma unroll 4
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride) {
        const uint4 v = src[i];
        acc.x ^= v.x;
        acc.y ^= v.y;
        acc.z ^= v.z;
        acc.w ^= v.w;
    }
    out[blockIdx.x * 256 + threadIdx.x] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

// CH chains of 32-bit bitwise operations per lane, each step of a chain
// depending on two other chains: three-input XORs (v_bitop3_b32) when OP3,
// else two-input XORs (v_xor_b32). UNROLL steps of the iteration loop per
// back-edge, so that the loop's scalar bookkeeping shrinks against the VALU
// work. Every operation counts once.
template <int CH, bool OP3, int UNROLL>
__global__ __launch_bounds__(256) void valu_chain(uint32_t *out, int iters)
{
    uint32_t a[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k)
        a[k] = threadIdx.x * (k + 3) + blockIdx.x;
#pragma unroll UNROLL
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < CH; ++k) {
            if constexpr (OP3)
                a[k] = __builtin_amdgcn_bitop3_b32(a[k], a[(k + 1) % CH], a[(k + 3) % CH], 0x96);
            else
                a[k] ^= a[(k + 1) % CH];
        }
    }
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < CH; ++k)
        r ^= a[k];
    out[blockIdx.x * 256 + threadIdx.x] = r;
}

// Times one VALU variant at `blocks_per_cu` workgroups of 4 waves per CU (one
// wave per SIMD each) and prints lane-operations per second and per CU clock.
template <int CH, bool OP3, int UNROLL>
int run_valu(const char *what, uint32_t *d, int cus, int blocks_per_cu)
{
    const int grid = cus * blocks_per_cu, iters = 20000;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return 1;
    hipLaunchKernelGGL((valu_chain<CH, OP3, UNROLL>), dim3(grid), dim3(256), 0, 0, d, 16);
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL((valu_chain<CH, OP3, UNROLL>), dim3(grid), dim3(256), 0, 0, d, iters);
    (void)hipEventRecord(b, 0);
    if (hipEventSynchronize(b) != hipSuccess)
        return 1;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    const double ops = (double)grid * 256 * iters * CH;
    printf("%-40s %2d waves/SIMD %7.2f T ops/s %6.1f lane-ops/clk/CU\n", what, blocks_per_cu, ops / ms / 1e9,
           ops / (ms * 1e-3) / cus / 2.4e9);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return 0;
}

template <int MODE, int W>
int run(const char *what, uint32_t *d, int cus)
{
    const int grid = cus * 8;
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        return 1;
    hipLaunchKernelGGL((lds_probe<MODE, W>), dim3(grid), dim3(256), 0, 0, d, 10);
    (void)hipEventRecord(a, 0);
    hipLaunchKernelGGL((lds_probe<MODE, W>), dim3(grid), dim3(256), 0, 0, d, ITERS);
    (void)hipEventRecord(b, 0);
    if (hipEventSynchronize(b) != hipSuccess)
        return 1;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    const double bytes = (double)grid * 256 * ITERS * 16 * 4 * W;
    printf("%-40s %7.1f TB/s  %6.1f B/clk/CU\n", what, bytes / ms / 1e9, bytes / (ms * 1e-3) / cus / 2.4e9);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return 0;
}

}  // namespace

int main()
{
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, 0) != hipSuccess) {
        fprintf(stderr, "no HIP device\n");
        return 1;
    }
    printf("%s, %d CUs, %zu B LDS per workgroup\n", p.gcnArchName, p.multiProcessorCount, p.sharedMemPerBlock);
    uint32_t *d = nullptr;
    if (hipMalloc(&d, (size_t)p.multiProcessorCount * 8 * 256 * 4) != hipSuccess)
        return 1;
    const int cus = p.multiProcessorCount;
    int rc = 0;
    {   // HBM
        const uint64_t bytes = 4ull << 30;
        void *src = nullptr;
        if (hipMalloc(&src, bytes) != hipSuccess || hipMemset(src, 1, bytes) != hipSuccess)
            return 1;
        const int grid = cus * 8;
        hipEvent_t a, b;
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
        hipLaunchKernelGGL(hbm_read, dim3(grid), dim3(256), 0, 0, static_cast<const uint4 *>(src), bytes / 16, d);
        (void)hipEventRecord(a, 0);
        for (int i = 0; i < 5; ++i)
            hipLaunchKernelGGL(hbm_read, dim3(grid), dim3(256), 0, 0, static_cast<const uint4 *>(src), bytes / 16,
                               d);
        (void)hipEventRecord(b, 0);
        if (hipEventSynchronize(b) != hipSuccess)
            return 1;
        float ms = 0;
        (void)hipEventElapsedTime(&ms, a, b);
        printf("%-40s %7.1f GB/s (4 GiB, 5 passes)\n", "HBM streaming read", 5.0 * bytes / ms / 1e6);
        (void)hipFree(src);
    }
    // VALU: the first line is the figure the read kernels are compared with
    // (eight chains of three-input XORs, 8 waves per SIMD); the others vary
    // the operation, the chains per lane and the waves per SIMD.
    rc |= run_valu<8, true, 1>("v_bitop3_b32, 8 chains", d, cus, 8);
    rc |= run_valu<16, true, 4>("v_bitop3_b32, 16 chains, unroll 4", d, cus, 8);
    rc |= run_valu<16, false, 4>("v_xor_b32, 16 chains, unroll 4", d, cus, 8);
    for (int w : {1, 2, 4})
        rc |= run_valu<16, true, 4>("v_bitop3_b32, 16 chains, unroll 4", d, cus, w);
    rc |= run<0, 1>("ds_read_b32 (4 B per lane)", d, p.multiProcessorCount);
    rc |= run<0, 2>("ds_read_b64 (8 B per lane)", d, p.multiProcessorCount);
    rc |= run<0, 4>("ds_read_b128 (16 B per lane)", d, p.multiProcessorCount);
    rc |= run<1, 1>("ds_write_b32 (4 B per lane)", d, p.multiProcessorCount);
    rc |= run<1, 2>("ds_write_b64 (8 B per lane)", d, p.multiProcessorCount);
    rc |= run<1, 4>("ds_write_b128 (16 B per lane)", d, p.multiProcessorCount);
    rc |= run<2, 4>("4 ds_read_b128 : 1 ds_write_b128", d, p.multiProcessorCount);
    rc |= run<3, 4>("paired lookups (2 adds + 4 xor3 / 2 reads)", d, p.multiProcessorCount);
    rc |= run<4, 4>("paired lookups + 1/8 ds_write_b128", d, p.multiProcessorCount);
    (void)hipFree(d);
    return rc;
}

// LDS bandwidth probe for gfx950: aggregate LDS throughput of the access
// patterns the Four-Russians kernels use. Every lane of a wave touches
// consecutive bytes of one contiguous row slice (64 lanes x W dwords), so the
// accesses are free of bank conflicts; all indices stay inside the 64 KiB
// array. Reported per CU and clock at 2.4 GHz; these figures set the LDS
// roofline of the table kernels.
//
//   ./paper_2001_08250_amd/lds_probe
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>

namespace {

constexpr int N = 16384;  // dwords = 64 KiB
constexpr int ITERS = 2000;

// MODE 0: reads of W dwords per lane; MODE 1: 16-byte writes; MODE 2: four
// 16-byte reads per 16-byte write (a table lookup phase with a build share).
template <int MODE, int W>
__global__ __launch_bounds__(256) void lds_probe(uint32_t *out, int iters)
{
    __shared__ uint32_t s[N];
    for (int i = threadIdx.x; i < N; i += 256)
        s[i] = i * 2654435761u;
    __syncthreads();
    uint4 acc = make_uint4(threadIdx.x, 1u, 2u, 3u);
    const int base = threadIdx.x * W;  // < 1024 dwords
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int o = base + k * 256 * W;  // <= 1020 + 15 * 1024 = 16380, +3 < N
            if constexpr (MODE == 0) {
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
    int rc = run<0, 1>("ds_read_b32 (4 B per lane)", d, p.multiProcessorCount);
    rc |= run<0, 2>("ds_read_b64 (8 B per lane)", d, p.multiProcessorCount);
    rc |= run<0, 4>("ds_read_b128 (16 B per lane)", d, p.multiProcessorCount);
    rc |= run<1, 4>("ds_write_b128 (16 B per lane)", d, p.multiProcessorCount);
    rc |= run<2, 4>("4 ds_read_b128 : 1 ds_write_b128", d, p.multiProcessorCount);
    (void)hipFree(d);
    return rc;
}

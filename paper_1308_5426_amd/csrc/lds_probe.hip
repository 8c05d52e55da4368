// lds_probe.hip -- achievable LDS read bandwidth (see include/ptmi_probe.h).
#include <hip/hip_runtime.h>

#include "ptmi_probe.h"

namespace {

constexpr int kBufBytes = 64 * 1024;

__global__ __launch_bounds__(1024) void k_lds_read(int iters, uint4 *sink)
{
    __shared__ uint4 buf[kBufBytes / sizeof(uint4)];
    constexpr int n = kBufBytes / sizeof(uint4);
    for (int e = threadIdx.x; e < n; e += blockDim.x) buf[e] = make_uint4(e, e + 1, e + 2, e + 3);
    __syncthreads();
    uint4 acc = make_uint4(0, 0, 0, 0);
    int at = threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll 8
        for (int k = 0; k < 8; ++k) {
            const uint4 v = buf[(at + k * blockDim.x) & (n - 1)];
            acc.x ^= v.x; acc.y ^= v.y; acc.z ^= v.z; acc.w ^= v.w;
        }
        at = (at + 8 * blockDim.x) & (n - 1);
    }
    if ((acc.x ^ acc.y ^ acc.z ^ acc.w) == 0x12345678u) sink[blockIdx.x] = acc;
}

}  // namespace

extern "C" int ptmi_lds_read_bandwidth(int32_t blocks, int32_t threads, int32_t iters, double *bytes_per_s)
{
    if (blocks < 1 || threads < 1 || threads > 1024 || iters < 1 || !bytes_per_s) return -1;
    uint4 *sink = nullptr;
    hipEvent_t e0, e1;
    if (hipMalloc(&sink, sizeof(uint4) * blocks) != hipSuccess) return -2;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(threads), 0, 0, iters, sink);  // warm-up
    if (hipEventRecord(e0, 0) != hipSuccess) return -4;
    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(threads), 0, 0, iters, sink);
    if (hipEventRecord(e1, 0) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -5;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -6;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    const double bytes = static_cast<double>(blocks) * threads * iters * 8.0 * sizeof(uint4);
    *bytes_per_s = bytes / (static_cast<double>(ms) * 1e-3);
    return 0;
}

// lds_probe.hip -- achievable LDS read bandwidth, and the field update alone
// (see include/ptmi_probe.h).
#include <hip/hip_runtime.h>

#include "ptmi_probe.h"
#include "sweep.hpp"  // the sweep kernel's own flush

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

constexpr int kReplayThreads = 256;

// The field update alone: a flip sequence applied window by window (64 flips
// at a time) to an FP64 field table in LDS by the sweep kernel's flush, with
// its doubled coupling row and coefficient table laid out as the sweep kernel
// lays them out.  Every workgroup replays the whole sequence on its own copy;
// workgroup 0 writes its final table.
__global__ __launch_bounds__(kReplayThreads) void k_flush_replay(int L, int q, int jlen, const double *J,
                                                                 const double *h0, const uint32_t *words,
                                                                 int64_t nwords, int reps, double *h_out)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double *Jl = reinterpret_cast<double *>(lds);  // [jlen]
    double *hl = Jl + jlen;                        // [q][L]
    double *ct = hl + static_cast<size_t>(q) * L;  // [256]
    uint32_t *pend = reinterpret_cast<uint32_t *>(ct + 256);
    for (int k = threadIdx.x; k < jlen; k += blockDim.x) Jl[k] = J[k % L];
    for (int e = threadIdx.x; e < q * L; e += blockDim.x) hl[e] = h0[e];
    for (int e = threadIdx.x; e < 256; e += blockDim.x) ct[e] = ptmi::flip_coef<double>(e & 3, (e >> 2) & 15, (e >> 2) >> 4);
    __syncthreads();
    ptmi::Inst P{};
    P.L = L;
    P.q = q;
    ptmi::Walker<double> W{};
    W.J = Jl;
    W.h = hl;
    W.ctab = ct;
    W.pend = pend;
    double part = 0.0;  // FP32 tables only
    for (int r = 0; r < reps; ++r) {
        for (int64_t p0 = 0; p0 < nwords; p0 += ptmi::kWave) {
            const int np = static_cast<int>(nwords - p0 < ptmi::kWave ? nwords - p0 : ptmi::kWave);
            if (threadIdx.x < ptmi::kWave) pend[threadIdx.x] = static_cast<int>(threadIdx.x) < np ? words[p0 + threadIdx.x] : ptmi::kNoFlip;
            __syncthreads();
            ptmi::flush_window<double, 4, true>(P, W, np, part, threadIdx.x, blockDim.x, q);  // every row stored
            __syncthreads();
        }
    }
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < q * L; e += blockDim.x) h_out[e] = hl[e];
}

// Issue rate of independent wave64 VALU instructions: every thread keeps 16
// accumulators and updates each `iters` times with one FMA of the kind (0:
// FP64, 1: FP32), with the multiplier 1 and the addend c from the host, so the
// results are exact and known: thread 0 of workgroup 0 writes the sum of its
// accumulators.
template <int K>
__global__ __launch_bounds__(1024) void k_valu(int iters, double bd, double cd, float bf, float cf, double *sum_out)
{
    double ad[16];
    float af[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        ad[k] = k;
        af[k] = static_cast<float>(k);
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if constexpr (K == 0) ad[k] = fma(ad[k], bd, cd);
            if constexpr (K == 1) af[k] = fmaf(af[k], bf, cf);
        }
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += K == 0 ? ad[k] : static_cast<double>(af[k]);
    if (blockIdx.x == 0 && threadIdx.x == 0) *sum_out = s;
}

}  // namespace

extern "C" int ptmi_valu_issue_rate(int32_t kind, int32_t blocks, int32_t threads, int32_t iters, double *ms_out,
                                    double *sum_out)
{
    if (kind < 0 || kind > 1 || blocks < 1 || threads < 64 || threads > 1024 || threads % 64 || iters < 1 ||
        iters > (1 << 20) || !ms_out || !sum_out)
        return -1;
    double *dsum = nullptr;
    if (hipMalloc(&dsum, sizeof(double)) != hipSuccess) return -3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -5;
    auto launch = [&](int n) {
        if (kind == 0)
            hipLaunchKernelGGL(k_valu<0>, dim3(blocks), dim3(threads), 0, 0, n, 1.0, 1.0, 1.0f, 1.0f, dsum);
        else
            hipLaunchKernelGGL(k_valu<1>, dim3(blocks), dim3(threads), 0, 0, n, 1.0, 1.0, 1.0f, 1.0f, dsum);
    };
    float ms = 0.f;
    if (!rc) {
        launch(16);  // warm-up
        if (hipEventRecord(e0, 0) != hipSuccess) rc = -6;
    }
    if (!rc) {
        launch(iters);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = -6;
    }
    if (!rc && hipMemcpy(sum_out, dsum, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess) rc = -7;
    *ms_out = ms;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dsum);
    return rc;
}

extern "C" int ptmi_flush_replay(int32_t L, int32_t q, const double *jstar, const double *h0, const uint32_t *words,
                                 int64_t nwords, int32_t workgroups, int32_t reps, double *h_out, double *ms_out)
{
    if (L < 2 || L > 65535 || q < 2 || q > 4 || !jstar || !h0 || (nwords > 0 && !words) || nwords < 0 ||
        workgroups < 1 || reps < 1 || !h_out || !ms_out)
        return -1;
    for (int64_t k = 0; k < nwords; ++k) {  // every word names a site and two states of this table
        const uint32_t w = words[k];
        if (static_cast<int>(w & 0xFFFFu) >= L || static_cast<int>((w >> 16) & 15u) >= q ||
            static_cast<int>((w >> 20) & 15u) >= q)
            return -1;
    }
    const int span = kReplayThreads * ptmi::kFlushM;
    const int jlen = L + (L + span - 1) / span * span;
    const size_t lds = sizeof(double) * (static_cast<size_t>(jlen) + static_cast<size_t>(q) * L + 256) +
                       sizeof(uint32_t) * ptmi::kWave;
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return -2;
    if (lds > static_cast<size_t>(lds_max)) return -1;
    if (hipFuncSetAttribute(reinterpret_cast<const void *>(&k_flush_replay),
                            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return -2;
    double *dJ = nullptr, *dh0 = nullptr, *dout = nullptr;
    uint32_t *dw = nullptr;
    const size_t hb = sizeof(double) * static_cast<size_t>(q) * L;
    int rc = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipMalloc(&dJ, sizeof(double) * L) != hipSuccess || hipMalloc(&dh0, hb) != hipSuccess ||
        hipMalloc(&dout, hb) != hipSuccess || hipMalloc(&dw, sizeof(uint32_t) * (nwords > 0 ? nwords : 1)) != hipSuccess)
        rc = -3;
    if (!rc && (hipMemcpy(dJ, jstar, sizeof(double) * L, hipMemcpyHostToDevice) != hipSuccess ||
                hipMemcpy(dh0, h0, hb, hipMemcpyHostToDevice) != hipSuccess ||
                (nwords > 0 && hipMemcpy(dw, words, sizeof(uint32_t) * nwords, hipMemcpyHostToDevice) != hipSuccess)))
        rc = -4;
    if (!rc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) rc = -5;
    if (!rc) {
        hipLaunchKernelGGL(k_flush_replay, dim3(workgroups), dim3(kReplayThreads), lds, 0, L, q, jlen, dJ, dh0, dw,
                           nwords, 1, dout);  // warm-up
        float ms = 0.f;
        if (hipEventRecord(e0, 0) != hipSuccess) rc = -6;
        if (!rc) {
            hipLaunchKernelGGL(k_flush_replay, dim3(workgroups), dim3(kReplayThreads), lds, 0, L, q, jlen, dJ, dh0,
                               dw, nwords, reps, dout);
            if (hipGetLastError() != hipSuccess || hipEventRecord(e1, 0) != hipSuccess ||
                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                rc = -6;
        }
        if (!rc && hipMemcpy(h_out, dout, hb, hipMemcpyDeviceToHost) != hipSuccess) rc = -7;
        *ms_out = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(dJ);
    (void)hipFree(dh0);
    (void)hipFree(dout);
    (void)hipFree(dw);
    return rc;
}

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

// device_common.hpp -- gfx950 device helpers: counter-based random stream,
// wave/workgroup reductions, the Hurwitz zeta function and the J* kernel.
//
// Paper: section 2, eqs. 5-7 (periodic couplings via Hurwitz zeta).  The
// paper evaluated J* on the CPU with a library zeta and copied it to the
// device; here the table is built on the GPU in FP64 by its own kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ptmi {

constexpr int kWave = 64;
constexpr int kQMax = 16;
constexpr double kBand = 1e-9;

// Lanes of the wave where p holds; the compare feeding it stays a lane mask.
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw; SC'11): ten rounds of two
// 32x32->64 multiplies with the key advanced by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
    constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
    constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
        const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

// u in (0,1) from 52 bits: (b + 1/2) * 2^-52, exact in FP64, never 0 or 1.
__device__ __forceinline__ double open_unit(uint32_t hi, uint32_t lo)
{
    const uint64_t b = (static_cast<uint64_t>(hi) << 20) | static_cast<uint64_t>(lo >> 12);
    return (static_cast<double>(b) + 0.5) * 0x1p-52;
}

// ---------------------------------------------------------------------------
// Reductions.  Lane 0 of each wave publishes its partial; every thread then
// sums the wave partials in the same order, so all threads get the same
// (deterministic) value.  `red` is LDS with room for blockDim.x/64 doubles.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

__device__ __forceinline__ double block_sum(double v, double *red)
{
    v = wave_sum(v);
    const int nw = blockDim.x / kWave;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += red[k];
    return t;
}

// ---------------------------------------------------------------------------
// Hurwitz zeta zeta(s, a) = sum_{k>=0} (k+a)^-s (eq. 7), s > 1, a > 0.
// Direct sum of the first 12 terms; the rest by Euler-Maclaurin with the
// coefficients B_2j/(2j)! for j = 1..9 (DLMF 25.11, 24.2).
// ---------------------------------------------------------------------------
__device__ double hurwitz_zeta(double s, double a)
{
    constexpr int kN = 12;
    double acc = 0.0;
    for (int k = kN - 1; k >= 0; --k) acc += pow(a + static_cast<double>(k), -s);
    const double x = a + static_cast<double>(kN);
    const double xs = pow(x, -s);
    acc += x * xs / (s - 1.0) + 0.5 * xs;
    // B_2j / (2j)!
    const double c[9] = {1.0 / 12.0,
                         -1.0 / 720.0,
                         1.0 / 30240.0,
                         -1.0 / 1209600.0,
                         1.0 / 47900160.0,
                         -691.0 / 1307674368000.0,
                         1.0 / 74724249600.0,
                         -3617.0 / 10670622842880000.0,
                         43867.0 / 5109094217170944000.0};
    const double ix2 = 1.0 / (x * x);
    double p = s * xs / x;  // s (s+1)..(s+2j-2) x^-(s+2j-1), j = 1
    for (int j = 0; j < 9; ++j) {
        acc += c[j] * p;
        const double m = s + 2.0 * j + 1.0;  // next two rising factors
        p *= m * (m + 1.0) * ix2;
    }
    return acc;
}

// J*(r) for 1 <= r <= L/2 by eq. 6, mirrored to L - r (J*(r) = J*(L-r));
// J*(0) = 0 (the self term i = j is excluded from eq. 2).
__device__ __forceinline__ void jstar_entry(int32_t L, double sigma, int r, double *J64, float *J32)
{
    double v = 0.0;
    if (r > 0) {
        const double s = 1.0 + sigma;
        const double t = static_cast<double>(r) / static_cast<double>(L);
        v = pow(static_cast<double>(r), -s) +
            pow(static_cast<double>(L), -s) * (hurwitz_zeta(s, 1.0 + t) + hurwitz_zeta(s, 1.0 - t));
    }
    J64[r] = v;
    J32[r] = static_cast<float>(v);
    if (r > 0 && L - r != r) {
        J64[L - r] = v;
        J32[L - r] = static_cast<float>(v);
    }
}

// Zero fill of device memory (used instead of a memset node, so the call can
// also be captured in a graph): 8-byte words when pointer and size allow,
// bytes otherwise.
static __global__ void k_zero(unsigned char *__restrict__ p, size_t n)
{
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t t0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if ((reinterpret_cast<uintptr_t>(p) & 7u) == 0 && (n & 7u) == 0) {
        uint64_t *w = reinterpret_cast<uint64_t *>(p);
        for (size_t e = t0; e < n / 8; e += stride) w[e] = 0ull;
    } else {
        for (size_t e = t0; e < n; e += stride) p[e] = 0;
    }
}

static __global__ void k_jstar(int32_t L, double sigma, double *__restrict__ J64, float *__restrict__ J32)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r <= L / 2) jstar_entry(L, sigma, r, J64, J32);
}

}  // namespace ptmi

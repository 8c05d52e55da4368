// Host-side helper for the oracle's Philox pin: evaluates rocRAND's
// philox4x32_10 engine (its __host__ path, no GPU needed) at given
// counters and keys.  rocRAND's engine(seed, subsequence, offset) places
// offset/4 in counter words 0-1 and the subsequence in words 2-3, with the
// key taken from the 64-bit seed.  Reads lines "c0 c1 c2 c3 k0 k1" (hex),
// prints "o0 o1 o2 o3" (hex).
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        const unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        const unsigned long long sub = ((unsigned long long)c3 << 32) | c2;
        const unsigned long long off = 4ULL * (((unsigned long long)c1 << 32) | c0);
        rocrand_device::philox4x32_10_engine e(seed, sub, off);
        const uint4 r = e.next4();
        std::printf("%08x %08x %08x %08x\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}

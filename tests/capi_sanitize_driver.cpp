// Host-side calls of the C ABI that touch no device (defaults, sizing,
// argument refusals, checkpoint checks), in a build of the host runtime with
// AddressSanitizer and UndefinedBehaviorSanitizer on its host code.  Built and
// run by tests/test_capi_sanitize.py without a GPU; exits 0 when every check
// passes.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "ptmi.h"

#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed: %s (line %d): %s\n", #c, __LINE__, pt_last_error()); \
            return 1;                                                          \
        }                                                                      \
    } while (0)

// A checkpoint in the library's layout: header, T, spins (0-based), perm, six
// moment sums and four counter arrays per slot.
static std::vector<unsigned char> checkpoint(int32_t L, int32_t q, int32_t R, const std::vector<uint8_t> &spins,
                                             const std::vector<int32_t> &perm)
{
    std::vector<unsigned char> b;
    auto put = [&](const void *p, size_t n) {
        const auto *c = static_cast<const unsigned char *>(p);
        b.insert(b.end(), c, c + n);
    };
    const uint32_t magic = 0x50544D49u, version = 1u;
    const int32_t prec = 0, init = 0, refresh = 0;
    const uint64_t seed = 1234;
    const double sigma = 0.5;
    const int64_t z = 0;
    put(&magic, 4); put(&version, 4); put(&L, 4); put(&q, 4); put(&R, 4); put(&prec, 4); put(&init, 4);
    put(&refresh, 4); put(&seed, 8); put(&sigma, 8); put(&z, 8); put(&z, 8); put(&z, 8);
    for (int k = 0; k < R; ++k) {
        const double t = 1.0 + k;
        put(&t, 8);
    }
    put(spins.data(), spins.size());
    put(perm.data(), 4 * perm.size());
    const std::vector<double> sums(6 * R, 0.0);
    const std::vector<int64_t> counts(4 * R, 0);
    put(sums.data(), 8 * sums.size());
    put(counts.data(), 8 * counts.size());
    return b;
}

int main()
{
    pt_options opt;
    pt_default_options(&opt);
    CHECK(opt.precision == PT_PREC_F64);
    size_t n64 = 0, n32 = 0, ni = 0;
    CHECK(pt_workspace_size(1024, 3, 64, &opt, &n64) == PT_OK);
    opt.precision = PT_PREC_F32;
    CHECK(pt_workspace_size(1024, 3, 64, &opt, &n32) == PT_OK);
    opt.precision = PT_PREC_I32;
    CHECK(pt_workspace_size(1024, 3, 64, &opt, &ni) == PT_OK);
    CHECK(n32 < n64 && ni == n32);
    CHECK(pt_workspace_size(1, 3, 64, &opt, &n64) == PT_EINVAL);
    CHECK(pt_workspace_size(10, 17, 64, &opt, &n64) == PT_EINVAL);
    CHECK(std::strlen(pt_last_error()) > 0);

    pt_ctx *ctx = nullptr;
    const double T2[2] = {2.0, 1.0}, Tok[2] = {1.0, 2.0};
    CHECK(pt_init(&ctx, 10, 3, 0.5, T2, 2, 1, nullptr) == PT_EINVAL && !ctx);  // descending ladder
    CHECK(pt_init(&ctx, 10, 3, 0.0, Tok, 2, 1, nullptr) == PT_EINVAL && !ctx);  // sigma 0
    pt_default_options(&opt);
    opt.precision = 3;
    CHECK(pt_init(&ctx, 10, 3, 0.5, Tok, 2, 1, &opt) == PT_EINVAL && !ctx);
    pt_default_options(&opt);
    opt.precision = PT_PREC_I32;
    opt.placement = PT_PLACE_DIRECT;  // direct sums keep no table: no int form
    CHECK(pt_init(&ctx, 10, 3, 0.5, Tok, 2, 1, &opt) == PT_EINVAL && !ctx);
    CHECK(pt_sweep(nullptr, 1) == PT_EINVAL);
    CHECK(pt_server_cancel(nullptr, 0) == PT_EINVAL);

    // the allocation-free entry point refuses on the host
    std::vector<double> T(128);
    for (int k = 0; k < 128; ++k) T[k] = 0.5 + 0.01 * k;
    CHECK(pt_run_static(1, 3, 0.5, T.data(), 4, 1, 1, 1, nullptr, nullptr, nullptr, nullptr) == PT_EINVAL);
    CHECK(pt_run_static(65535, 16, 0.5, T.data(), 128, 1, 1, 1, nullptr, nullptr, nullptr, nullptr) == PT_EINVAL);

    // batch and server sizing
    pt_job_desc jobs[2] = {{64, 3, 0.5, Tok, 2, 7, 10, 1, PT_INIT_RANDOM},
                           {1000, 10, 0.3, T.data(), 32, 8, 5, 2, PT_INIT_ORDERED}};
    size_t bb = 0, sb = 0;
    CHECK(pt_batch_workspace_size(jobs, 2, nullptr, &bb) == PT_OK && bb > 0);
    jobs[1].exchange_every = 0;
    CHECK(pt_batch_workspace_size(jobs, 2, nullptr, &bb) == PT_EINVAL);
    CHECK(pt_batch_workspace_size(nullptr, 0, nullptr, &bb) == PT_EINVAL);
    CHECK(pt_server_workspace_size(1 << 20, 16, &sb) == PT_OK && sb > (1u << 20));
    CHECK(pt_server_workspace_size(1 << 20, 0, &sb) == PT_EINVAL);

    // corrupt checkpoints are refused before any device call
    const int32_t L = 16, q = 3, R = 4;
    std::vector<uint8_t> spins(static_cast<size_t>(R) * L, 0);
    std::vector<int32_t> perm = {0, 1, 2, 3};
    for (int kind = 0; kind < 6; ++kind) {
        std::vector<uint8_t> s = spins;
        std::vector<int32_t> p = perm;
        int32_t qq = q;
        if (kind == 0) s[2 * L + 7] = q;        // a spin equal to q
        if (kind == 1) s[0] = 255;              // a spin far out of range
        if (kind == 2) p = {0, 1, 1, 3};        // perm with a duplicate
        if (kind == 3) p = {0, 1, 2, 4};        // perm out of range
        if (kind == 4) qq = 99;                 // bad sizes in the header
        std::vector<unsigned char> blob = checkpoint(L, qq, R, s, p);
        if (kind == 5) blob.resize(blob.size() - 8);  // truncated
        pt_ctx *c = nullptr;
        CHECK(pt_load(&c, blob.data(), blob.size(), nullptr) == PT_EINVAL && !c);
    }
    std::vector<unsigned char> junk(3, 0);
    pt_ctx *c = nullptr;
    CHECK(pt_load(&c, junk.data(), junk.size(), nullptr) == PT_EINVAL && !c);
    CHECK(pt_load(&c, nullptr, 0, nullptr) == PT_EINVAL && !c);
    std::puts("ok");
    return 0;
}

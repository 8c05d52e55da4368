/* Exercises every entry point of the oracle (oracle/orc.c) on small and edge
 * cases, so that a build with AddressSanitizer and UndefinedBehaviorSanitizer
 * reports any out-of-bounds access, leak or undefined operation.  Built and
 * run by tests/test_oracle_sanitize.py; exits 0 when every check passes. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

#define CHECK(c)                                                  \
    do {                                                          \
        if (!(c)) {                                               \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                             \
        }                                                         \
    } while (0)

static int run_pt(int L, int q, int R, int mode, int init, int threads, int every)
{
    double *T = malloc(sizeof(double) * R);
    for (int k = 0; k < R; ++k) T[k] = 0.3 * pow(10.0, R > 1 ? (double)k / (R - 1) : 0.0);
    orc_pt *p = orc_pt_create(L, q, 0.5, T, R, 1234u + (uint64_t)L, init, mode);
    CHECK(p != NULL);
    orc_pt_set_threads(p, threads);
    orc_pt_record_series(p, 1);
    CHECK(orc_pt_run(p, 7, every) == 0);
    CHECK(orc_pt_sweep(p, 2) == 0);
    CHECK(orc_pt_exchange(p) == 0);
    uint8_t *s = malloc((size_t)R * L);
    int32_t *perm = malloc(sizeof(int32_t) * R);
    double *E = malloc(sizeof(double) * R);
    double *sum6 = malloc(sizeof(double) * 6 * R);
    int64_t *fa = malloc(sizeof(int64_t) * R), *fc = malloc(sizeof(int64_t) * R);
    int64_t *xa = malloc(sizeof(int64_t) * R), *xc = malloc(sizeof(int64_t) * R);
    int64_t c3[3];
    orc_pt_get_spins(p, s);
    orc_pt_get_perm(p, perm);
    orc_pt_get_energy(p, E);
    orc_pt_get_stats(p, sum6, fa, fc, xa, xc, c3);
    for (int w = 0; w < R; ++w) {
        CHECK(fabs(orc_pt_energy_full(p, w) - E[w]) <= 1e-9 * (1.0 + fabs(E[w])));
        for (int j = 0; j < L; ++j) CHECK(s[(size_t)w * L + j] >= 1 && s[(size_t)w * L + j] <= q);
    }
    const int64_t n = orc_pt_series_len(p);
    CHECK(n == 9);
    double *sE = malloc(sizeof(double) * (size_t)n * R), *sM = malloc(sizeof(double) * (size_t)n * R);
    orc_pt_get_series(p, sE, sM);
    /* replay a logged decision (adopted only inside the band: none here) */
    const int64_t mw = 0, mn = 0, mt = 0, em = 0, eg = 0, ek = 0;
    const int8_t md = 1, ed = 0;
    orc_pt_set_replay(p, 1, &mw, &mn, &mt, &md, 1, &em, &eg, &ek, &ed);
    CHECK(orc_pt_run(p, 3, 1) == 0);
    CHECK(orc_pt_banded_count(p) >= 0);
    /* spins set from outside: every state, then the fields and energy recomputed */
    for (size_t e = 0; e < (size_t)R * L; ++e) s[e] = (uint8_t)(1 + e % (size_t)q);
    orc_pt_set_spins(p, s);
    orc_pt_get_energy(p, E);
    for (int w = 0; w < R; ++w) CHECK(fabs(orc_pt_energy_full(p, w) - E[w]) <= 1e-9 * (1.0 + fabs(E[w])));
    orc_pt_free(p);
    free(T); free(s); free(perm); free(E); free(sum6); free(fa); free(fc); free(xa); free(xc); free(sE); free(sM);
    return 0;
}

int main(void)
{
    /* special functions */
    const double pi = 3.14159265358979323846;
    CHECK(fabs(orc_hurwitz_zeta(2.0, 1.0) - pi * pi / 6.0) < 1e-14);
    CHECK(isfinite(orc_hurwitz_zeta(1.05, 0.5)) && isfinite(orc_hurwitz_zeta(3.0, 1.999)));
    const int Ls[] = {2, 3, 64, 1001};
    for (size_t k = 0; k < sizeof Ls / sizeof Ls[0]; ++k) {
        const int L = Ls[k];
        double *J = malloc(sizeof(double) * L);
        CHECK(orc_jstar(L, 0.4, J) == 0);
        CHECK(J[0] == 0.0);
        uint8_t *s = malloc((size_t)L);
        int8_t *sig = malloc((size_t)L);
        for (int j = 0; j < L; ++j) {
            s[j] = (uint8_t)(1 + (j * 7) % 3);
            sig[j] = (int8_t)((j % 2) ? 1 : -1);
        }
        CHECK(isfinite(orc_energy(L, J, s)));
        CHECK(isfinite(orc_energy_ising(L, J, sig)));
        const double M = orc_magnetization(L, 3, s);
        CHECK(M >= 0.0 && M <= 1.0);
        double Ei = orc_energy_ising(L, J, sig);
        CHECK(orc_ising_sweeps(L, J, sig, 0.7, 99u, 0, 0, 3, &Ei) == 0);
        free(J); free(s); free(sig);
    }
    uint32_t ctr[4] = {0, 1, 2, 3}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    /* parallel tempering: both energy modes, both starts, q from 2 to 16, one
     * replica and several, one thread and several */
    CHECK(run_pt(2, 2, 1, 0, 0, 1, 1) == 0);
    CHECK(run_pt(3, 16, 3, 1, 1, 2, 2) == 0);
    CHECK(run_pt(65, 3, 4, 0, 0, 2, 1) == 0);
    CHECK(run_pt(65, 5, 4, 1, 0, 3, 3) == 0);
    CHECK(run_pt(130, 10, 5, 1, 1, 1, 1) == 0);
    puts("ok");
    return 0;
}

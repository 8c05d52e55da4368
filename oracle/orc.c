/*
 * orc.c -- plain FP64 CPU oracle for parallel tempering of the 1D
 * long-range q-state Potts ring.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares
 * no code, header, table or constant with the GPU library.
 *
 * Every function is written from the paper's definitions:
 *   eq. 1      spins s_i in 1..q
 *   eqs. 2-3   H = -sum J_ij delta(s_i, s_j); each unordered pair counted once
 *   eqs. 4-7   J(r) = r^-(1+sigma); periodic J*(r) = sum_n J(r + nL), written
 *              with two Hurwitz zeta values; zeta(s,a) = sum_k (k+a)^-s
 *   eq. 8      Metropolis single-spin flip, accept with min(1, exp(-beta dE))
 *   eq. 9      replica exchange, accept with min(1, exp((E_i-E_j)(beta_i-beta_j)))
 *   sec. 4.2   exchange in two stages: pairs (i, i+1) with i even, then odd
 *   eq. 10     M = (q Nmax / N - 1) / (q - 1)
 *
 * Readings where the paper is silent (proposal, site choice, random stream,
 * tie rule, recording order) are those listed in the design notes: the new
 * state is uniform over the q-1 other states, the site is uniform, x = beta
 * dE + ln u is accepted iff x < 0, observables are recorded after a sweep and
 * before the exchange that follows it.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Hurwitz zeta (eq. 7): the first N terms summed directly, the remainder   */
/* sum_{k>=N} (k+a)^-s by the Euler-Maclaurin formula                       */
/*   int_N^inf + f(N)/2 - sum_j B_2j/(2j)! f^(2j-1)(N),                      */
/* with f(k) = (k+a)^-s, f^(m)(x) = (-1)^m s(s+1)..(s+m-1) x^-(s+m).        */
/* ------------------------------------------------------------------------ */
double orc_hurwitz_zeta(double s, double a)
{
    enum { NDIRECT = 16, NBERN = 10 };
    /* Bernoulli numbers B_2 .. B_20 as exact fractions. */
    static const double bern_num[NBERN] = {1, -1, 1, -1, 5, -691, 7, -3617, 43867, -174611};
    static const double bern_den[NBERN] = {6, 30, 42, 30, 66, 2730, 6, 510, 798, 330};
    double sum = 0.0;
    for (int k = 0; k < NDIRECT; ++k) sum += pow(a + k, -s);
    const double x = a + NDIRECT;
    sum += pow(x, 1.0 - s) / (s - 1.0); /* integral of (t)^-s from x to inf */
    sum += 0.5 * pow(x, -s);
    double fact = 1.0;             /* (2j)! */
    double rising = s;             /* s (s+1) ... (s+2j-2) */
    double xp = pow(x, -s - 1.0);  /* x^-(s+2j-1) */
    for (int j = 1; j <= NBERN; ++j) {
        fact *= (double)(2 * j - 1) * (double)(2 * j);
        /* -B_2j/(2j)! f^(2j-1)(x) = +B_2j/(2j)! s..(s+2j-2) x^-(s+2j-1) */
        sum += (bern_num[j - 1] / bern_den[j - 1]) / fact * rising * xp;
        rising *= (s + 2.0 * j - 1.0) * (s + 2.0 * j);
        xp /= x * x;
    }
    return sum;
}

/* eq. 6: J*(r) = r^-s + L^-s [zeta(s, 1 + r/L) + zeta(s, 1 - r/L)], s = 1 + sigma. */
int orc_jstar(int32_t L, double sigma, double *J)
{
    if (L < 2 || !(sigma > 0.0) || !J) return -1;
    const double s = 1.0 + sigma;
    const double Ls = pow((double)L, -s);
    J[0] = 0.0;
    for (int32_t r = 1; r < L; ++r) {
        const double x = (double)r / (double)L;
        J[r] = pow((double)r, -s) + Ls * (orc_hurwitz_zeta(s, 1.0 + x) + orc_hurwitz_zeta(s, 1.0 - x));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10, from the round function published by Salmon et al.:      */
/*   (hi0,lo0) = M0*c0, (hi1,lo1) = M1*c2,                                   */
/*   c' = (hi1^c1^k0, lo1, hi0^c3^k1, lo0); key bumped by (W0, W1)           */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n1 = (uint32_t)p1;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        const uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static uint32_t mulhi32(uint32_t x, uint32_t n) { return (uint32_t)(((uint64_t)x * n) >> 32); }

/* Uniform in (0,1): 52 random bits b, u = (b + 1/2) 2^-52 (exact in FP64). */
static double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t b = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)b + 0.5) * 0x1p-52;
}

static void stream(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t out[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* Energy and magnetisation                                                  */
/* ------------------------------------------------------------------------ */
double orc_energy(int32_t L, const double *J, const uint8_t *s)
{
    double e = 0.0;
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = i + 1; j < L; ++j)
            if (s[i] == s[j]) e -= J[j - i];
    return e;
}

double orc_energy_ising(int32_t L, const double *J, const int8_t *sig)
{
    double e = 0.0;
    for (int32_t i = 0; i < L; ++i)
        for (int32_t j = i + 1; j < L; ++j) e -= J[j - i] * (double)sig[i] * (double)sig[j];
    return e;
}

double orc_magnetization(int32_t L, int32_t q, const uint8_t *s)
{
    int32_t cnt[256];
    memset(cnt, 0, sizeof cnt);
    for (int32_t i = 0; i < L; ++i) cnt[s[i]]++;
    int32_t nmax = 0;
    for (int32_t k = 1; k <= q; ++k)
        if (cnt[k] > nmax) nmax = cnt[k];
    return ((double)q * (double)nmax / (double)L - 1.0) / (double)(q - 1);
}

/* ------------------------------------------------------------------------ */
/* Parallel tempering                                                        */
/* ------------------------------------------------------------------------ */
#define ORC_BAND 1e-9

struct orc_pt {
    int32_t L, q, R, mode, nthreads, record, wbase;
    uint64_t seed;
    int64_t sweeps, xsteps;
    double *J;      /* [L] */
    double *beta;   /* [R] by slot */
    uint8_t *s;     /* [R][L] by walker */
    double *h;      /* [R][q][L] field table (mode 1) */
    double *E;      /* [R] by walker */
    int32_t *perm;  /* slot -> walker */
    int32_t *slot;  /* walker -> slot */
    double *sum6;   /* [6][R] by slot */
    int64_t *fatt, *facc, *xatt, *xacc;
    int64_t samples, banded_met, banded_ex;
    double *serE, *serM;
    int64_t serlen, sercap;
    int64_t nmet, nex;
    int64_t *met_w, *met_n, *met_t, *ex_m, *ex_g, *ex_k;
    int8_t *met_dec, *ex_dec;
};

static void fields_from_spins(orc_pt *p, int32_t w)
{
    const int32_t L = p->L, q = p->q;
    double *h = p->h + (size_t)w * q * L;
    const uint8_t *s = p->s + (size_t)w * L;
    for (int32_t k = 0; k < q; ++k)
        for (int32_t j = 0; j < L; ++j) {
            double acc = 0.0;
            for (int32_t i = 0; i < L; ++i)
                if (i != j && s[i] == k + 1) acc += p->J[(j - i + L) % L];
            h[(size_t)k * L + j] = acc;
        }
}

orc_pt *orc_pt_create(int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed,
                      int32_t init, int32_t mode)
{
    return orc_pt_create_at(L, q, sigma, T, R, seed, init, mode, 0);
}

/* As orc_pt_create, with walker k of this object taking the random stream of
 * walker wbase + k (to follow selected walkers of a larger run). */
orc_pt *orc_pt_create_at(int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed,
                         int32_t init, int32_t mode, int32_t wbase)
{
    if (L < 2 || q < 2 || q > 255 || !(sigma > 0.0) || R < 1 || !T) return NULL;
    for (int32_t k = 0; k < R; ++k)
        if (!(T[k] > 0.0) || !isfinite(T[k])) return NULL;
    orc_pt *p = (orc_pt *)calloc(1, sizeof *p);
    p->L = L; p->q = q; p->R = R; p->mode = mode; p->seed = seed; p->nthreads = 1; p->wbase = wbase;
    p->J = (double *)malloc(sizeof(double) * L);
    orc_jstar(L, sigma, p->J);
    p->beta = (double *)malloc(sizeof(double) * R);
    for (int32_t k = 0; k < R; ++k) p->beta[k] = 1.0 / T[k];
    p->s = (uint8_t *)malloc((size_t)R * L);
    for (int32_t w = 0; w < R; ++w)
        for (int32_t j = 0; j < L; ++j) {
            uint8_t v = 1;
            if (init == 0) {
                uint32_t o[4];
                stream(seed, (uint32_t)j, 0u, (uint32_t)(wbase + w), 2u, o);
                v = (uint8_t)(1 + mulhi32(o[0], (uint32_t)q));
            }
            p->s[(size_t)w * L + j] = v;
        }
    p->E = (double *)malloc(sizeof(double) * R);
    if (mode == 1) p->h = (double *)malloc(sizeof(double) * (size_t)R * q * L);
    /* walkers are independent: their O(L^2) initial energies (and fields) are
       computed in parallel, each by the same sequential loop */
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t w = 0; w < R; ++w) {
        p->E[w] = orc_energy(L, p->J, p->s + (size_t)w * L);
        if (mode == 1) fields_from_spins(p, w);
    }
    p->perm = (int32_t *)malloc(sizeof(int32_t) * R);
    p->slot = (int32_t *)malloc(sizeof(int32_t) * R);
    for (int32_t k = 0; k < R; ++k) p->perm[k] = p->slot[k] = k;
    p->sum6 = (double *)calloc((size_t)6 * R, sizeof(double));
    p->fatt = (int64_t *)calloc(R, sizeof(int64_t));
    p->facc = (int64_t *)calloc(R, sizeof(int64_t));
    p->xatt = (int64_t *)calloc(R, sizeof(int64_t));
    p->xacc = (int64_t *)calloc(R, sizeof(int64_t));
    return p;
}

void orc_pt_free(orc_pt *p)
{
    if (!p) return;
    free(p->J); free(p->beta); free(p->s); free(p->h); free(p->E); free(p->perm); free(p->slot);
    free(p->sum6); free(p->fatt); free(p->facc); free(p->xatt); free(p->xacc);
    free(p->serE); free(p->serM);
    free(p->met_w); free(p->met_n); free(p->met_t); free(p->met_dec);
    free(p->ex_m); free(p->ex_g); free(p->ex_k); free(p->ex_dec);
    free(p);
}

void orc_pt_set_threads(orc_pt *p, int32_t n) { p->nthreads = n < 1 ? 1 : n; }
void orc_pt_record_series(orc_pt *p, int32_t on) { p->record = on; }

void orc_pt_set_replay(orc_pt *p, int64_t nmet, const int64_t *mw, const int64_t *mn, const int64_t *mt,
                       const int8_t *md, int64_t nex, const int64_t *em, const int64_t *eg,
                       const int64_t *ek, const int8_t *ed)
{
    free(p->met_w); free(p->met_n); free(p->met_t); free(p->met_dec);
    free(p->ex_m); free(p->ex_g); free(p->ex_k); free(p->ex_dec);
    p->nmet = nmet; p->nex = nex;
    p->met_w = (int64_t *)malloc(sizeof(int64_t) * (nmet + 1));
    p->met_n = (int64_t *)malloc(sizeof(int64_t) * (nmet + 1));
    p->met_t = (int64_t *)malloc(sizeof(int64_t) * (nmet + 1));
    p->met_dec = (int8_t *)malloc(nmet + 1);
    p->ex_m = (int64_t *)malloc(sizeof(int64_t) * (nex + 1));
    p->ex_g = (int64_t *)malloc(sizeof(int64_t) * (nex + 1));
    p->ex_k = (int64_t *)malloc(sizeof(int64_t) * (nex + 1));
    p->ex_dec = (int8_t *)malloc(nex + 1);
    for (int64_t e = 0; e < nmet; ++e) {
        p->met_w[e] = mw[e]; p->met_n[e] = mn[e]; p->met_t[e] = mt[e]; p->met_dec[e] = md[e];
    }
    for (int64_t e = 0; e < nex; ++e) {
        p->ex_m[e] = em[e]; p->ex_g[e] = eg[e]; p->ex_k[e] = ek[e]; p->ex_dec[e] = ed[e];
    }
}

static int replay_met(const orc_pt *p, int64_t w, int64_t n, int64_t t, int own)
{
    for (int64_t e = 0; e < p->nmet; ++e)
        if (p->met_w[e] == w && p->met_n[e] == n && p->met_t[e] == t) return p->met_dec[e] != 0;
    return own;
}

static int replay_ex(const orc_pt *p, int64_t m, int64_t g, int64_t k, int own)
{
    for (int64_t e = 0; e < p->nex; ++e)
        if (p->ex_m[e] == m && p->ex_g[e] == g && p->ex_k[e] == k) return p->ex_dec[e] != 0;
    return own;
}

/* One sweep (L attempts) of walker w at sweep index n; returns accepts. */
static int64_t sweep_walker(orc_pt *p, int32_t w, int64_t n, int64_t *banded)
{
    const int32_t L = p->L, q = p->q;
    const double beta = p->beta[p->slot[w]];
    uint8_t *s = p->s + (size_t)w * L;
    double *h = p->h ? p->h + (size_t)w * q * L : NULL;
    const double *J = p->J;
    int64_t acc = 0;
    for (int32_t t = 0; t < L; ++t) {
        uint32_t o[4];
        stream(p->seed, (uint32_t)t, (uint32_t)n, (uint32_t)(p->wbase + w), 0u, o);
        const int32_t i = (int32_t)mulhi32(o[0], (uint32_t)L);
        const int32_t k = 1 + (int32_t)mulhi32(o[1], (uint32_t)(q - 1));
        const double u = unit_open(o[2], o[3]);
        const int32_t a = s[i];
        const int32_t b = ((a - 1 + k) % q) + 1;
        double dE = 0.0;
        if (p->mode == 1) {
            dE = h[(size_t)(a - 1) * L + i] - h[(size_t)(b - 1) * L + i];
        } else {
            /* dE = sum_{j != i} J*(|i-j|) [delta(a, s_j) - delta(b, s_j)] */
            for (int32_t j = 0; j < L; ++j) {
                if (j == i) continue;
                if (s[j] == a) dE += J[(j - i + L) % L];
                else if (s[j] == b) dE -= J[(j - i + L) % L];
            }
        }
        const double x = beta * dE + log(u);
        int accept = x < 0.0;
        if (fabs(x) <= ORC_BAND) {
            ++*banded;
            accept = replay_met(p, w, n, t, accept);
        }
        if (accept) {
            if (h) {
                for (int32_t j = 0; j < L; ++j) {
                    const double Jr = J[(j - i + L) % L];
                    h[(size_t)(a - 1) * L + j] -= Jr;
                    h[(size_t)(b - 1) * L + j] += Jr;
                }
            }
            s[i] = (uint8_t)b;
            p->E[w] += dE;
            ++acc;
        }
    }
    return acc;
}

static void record(orc_pt *p)
{
    const int32_t R = p->R;
    if (p->record && p->serlen == p->sercap) {
        p->sercap = p->sercap ? 2 * p->sercap : 64;
        p->serE = (double *)realloc(p->serE, sizeof(double) * p->sercap * R);
        p->serM = (double *)realloc(p->serM, sizeof(double) * p->sercap * R);
    }
    for (int32_t k = 0; k < R; ++k) {
        const int32_t w = p->perm[k];
        const double e = p->E[w];
        const double m = orc_magnetization(p->L, p->q, p->s + (size_t)w * p->L);
        const double e2 = e * e, m2 = m * m;
        p->sum6[0 * R + k] += e;
        p->sum6[1 * R + k] += e2;
        p->sum6[2 * R + k] += e2 * e2;
        p->sum6[3 * R + k] += m;
        p->sum6[4 * R + k] += m2;
        p->sum6[5 * R + k] += m2 * m2;
        if (p->record) {
            p->serE[p->serlen * R + k] = e;
            p->serM[p->serlen * R + k] = m;
        }
    }
    if (p->record) p->serlen++;
    p->samples++;
}

int orc_pt_sweep(orc_pt *p, int64_t nsw)
{
    const int32_t R = p->R;
    int64_t *acc = (int64_t *)malloc(sizeof(int64_t) * R);
    for (int64_t it = 0; it < nsw; ++it) {
        const int64_t n = p->sweeps;
        int64_t banded = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(p->nthreads) reduction(+ : banded)
        for (int32_t w = 0; w < R; ++w) acc[w] = sweep_walker(p, w, n, &banded);
        p->banded_met += banded;
        for (int32_t w = 0; w < R; ++w) {
            p->fatt[p->slot[w]] += p->L;
            p->facc[p->slot[w]] += acc[w];
        }
        p->sweeps++;
        record(p);
    }
    free(acc);
    return 0;
}

int orc_pt_exchange(orc_pt *p)
{
    const int64_t m = p->xsteps;
    for (int32_t g = 0; g < 2; ++g) {
        for (int32_t k = g; k + 1 < p->R; k += 2) {
            const int32_t wa = p->perm[k], wb = p->perm[k + 1];
            const double delta = (p->E[wa] - p->E[wb]) * (p->beta[k] - p->beta[k + 1]);
            uint32_t o[4];
            stream(p->seed, (uint32_t)k, (uint32_t)m, (uint32_t)g, 1u, o);
            const double y = log(unit_open(o[0], o[1])) - delta;
            int accept = y < 0.0; /* ln u < (E_i - E_j)(beta_i - beta_j) */
            if (fabs(y) <= ORC_BAND) {
                p->banded_ex++;
                accept = replay_ex(p, m, g, k, accept);
            }
            p->xatt[k]++;
            if (accept) {
                p->perm[k] = wb; p->perm[k + 1] = wa;
                p->slot[wb] = k; p->slot[wa] = k + 1;
                p->xacc[k]++;
            }
        }
    }
    p->xsteps++;
    return 0;
}

int orc_pt_run(orc_pt *p, int64_t n, int32_t every)
{
    for (int64_t it = 0; it < n; ++it) {
        orc_pt_sweep(p, 1);
        if (every > 0 && (it + 1) % every == 0) orc_pt_exchange(p);
    }
    return 0;
}

void orc_pt_get_spins(const orc_pt *p, uint8_t *out) { memcpy(out, p->s, (size_t)p->R * p->L); }
void orc_pt_get_perm(const orc_pt *p, int32_t *out) { memcpy(out, p->perm, sizeof(int32_t) * p->R); }
void orc_pt_get_energy(const orc_pt *p, double *out) { memcpy(out, p->E, sizeof(double) * p->R); }

void orc_pt_get_stats(const orc_pt *p, double *sum6, int64_t *fatt, int64_t *facc, int64_t *xatt,
                      int64_t *xacc, int64_t *c3)
{
    const int32_t R = p->R;
    if (sum6) memcpy(sum6, p->sum6, sizeof(double) * 6 * R);
    if (fatt) memcpy(fatt, p->fatt, sizeof(int64_t) * R);
    if (facc) memcpy(facc, p->facc, sizeof(int64_t) * R);
    if (xatt) memcpy(xatt, p->xatt, sizeof(int64_t) * (R > 1 ? R - 1 : 0));
    if (xacc) memcpy(xacc, p->xacc, sizeof(int64_t) * (R > 1 ? R - 1 : 0));
    if (c3) { c3[0] = p->samples; c3[1] = p->banded_met; c3[2] = p->banded_ex; }
}

int64_t orc_pt_series_len(const orc_pt *p) { return p->serlen; }

void orc_pt_get_series(const orc_pt *p, double *E, double *M)
{
    if (E) memcpy(E, p->serE, sizeof(double) * p->serlen * p->R);
    if (M) memcpy(M, p->serM, sizeof(double) * p->serlen * p->R);
}

int64_t orc_pt_banded_count(const orc_pt *p) { return p->banded_met + p->banded_ex; }

double orc_pt_energy_full(const orc_pt *p, int32_t w) { return orc_energy(p->L, p->J, p->s + (size_t)w * p->L); }

void orc_pt_set_spins(orc_pt *p, const uint8_t *s)
{
    memcpy(p->s, s, (size_t)p->R * p->L);
    for (int32_t w = 0; w < p->R; ++w) {
        p->E[w] = orc_energy(p->L, p->J, p->s + (size_t)w * p->L);
        if (p->h) fields_from_spins(p, w);
    }
}

/* ------------------------------------------------------------------------ */
/* Separately written q = 2 path on +-1 spins.  The Potts flip at beta has  */
/* dE_Potts = dE_Ising / 2 (delta = (1 + sig_i sig_j)/2), so this path at    */
/* beta_ising = beta/2 must follow the same trajectory under the same draws.*/
/* ------------------------------------------------------------------------ */
int orc_ising_sweeps(int32_t L, const double *J, int8_t *sig, double beta_ising, uint64_t seed,
                     int32_t walker, int64_t sweep0, int64_t nsweeps, double *E_io)
{
    double E = E_io ? *E_io : 0.0;
    for (int64_t n = sweep0; n < sweep0 + nsweeps; ++n)
        for (int32_t t = 0; t < L; ++t) {
            uint32_t o[4];
            stream(seed, (uint32_t)t, (uint32_t)n, (uint32_t)walker, 0u, o);
            const int32_t i = (int32_t)mulhi32(o[0], (uint32_t)L);
            double local = 0.0;
            for (int32_t j = 0; j < L; ++j)
                if (j != i) local += J[(j - i + L) % L] * (double)sig[j];
            const double dE = 2.0 * (double)sig[i] * local;
            if (beta_ising * dE + log(unit_open(o[2], o[3])) < 0.0) {
                sig[i] = (int8_t)-sig[i];
                E += dE;
            }
        }
    if (E_io) *E_io = E;
    return 0;
}

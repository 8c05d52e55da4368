/*
 * orc.h -- plain FP64 CPU oracle for parallel tempering of the 1D long-range
 * q-state Potts ring (Boer, "GPU-based simulation of the long-range Potts
 * model via parallel tempering", Comput. Phys. Commun.).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: it is used by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark.  It shares no source, header, table or
 * constant with the GPU library.
 *
 * Conventions (paper section 2, eqs. 1-7; section 3, eqs. 8-9):
 *   spins are uint8 values 1..q (eq. 1);
 *   J[r] = J*(r) for r = 0..L-1 with J[0] = 0 (self term excluded, i != j);
 *   E(s) = -sum_{0<=i<j<L} J*(j-i) delta(s_i, s_j)   (each pair once);
 *   beta = 1/T (k_B = 1).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Hurwitz zeta zeta(s, a) = sum_{k>=0} (k+a)^-s, s > 1, a > 0 (eq. 7),
 * by direct summation plus an Euler-Maclaurin tail. */
double orc_hurwitz_zeta(double s, double a);

/* Periodic couplings J*(r) of eq. 5 via the closed form eq. 6, r = 1..L-1,
 * J[0] = 0.  Returns 0, or -1 on bad arguments. */
int orc_jstar(int32_t L, double sigma, double *J);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Energy (eq. 2, pairs once), Ising energy of +-1 spins with the same
 * couplings, and magnetisation (eq. 10). */
double orc_energy(int32_t L, const double *J, const uint8_t *s);
double orc_energy_ising(int32_t L, const double *J, const int8_t *sig);
double orc_magnetization(int32_t L, int32_t q, const uint8_t *s);

/* ---------------------------------------------------------------------- */
/* Parallel-tempering state machine.                                       */
/* mode 0: direct O(L) energy difference per attempt (the plain definition)*/
/* mode 1: FP64 local-field table, O(1) energy difference, O(L) update     */
/* init 0: uniform spins from the walker's stream; 1: all spins = 1        */
typedef struct orc_pt orc_pt;

orc_pt *orc_pt_create(int32_t L, int32_t q, double sigma, const double *T, int32_t R,
                      uint64_t seed, int32_t init, int32_t mode);
orc_pt *orc_pt_create_at(int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed,
                         int32_t init, int32_t mode, int32_t wbase);
void orc_pt_free(orc_pt *p);
void orc_pt_set_threads(orc_pt *p, int32_t nthreads);  /* OpenMP threads over walkers */
void orc_pt_record_series(orc_pt *p, int32_t on);       /* keep E, M per sweep and slot */

/* n sweeps (L attempts per walker each), observables recorded per slot
 * after each sweep; no exchange. */
int orc_pt_sweep(orc_pt *p, int64_t n);
/* One exchange step: even stage then odd stage. */
int orc_pt_exchange(orc_pt *p);
/* n sweeps with an exchange step after every `every`-th sweep. */
int orc_pt_run(orc_pt *p, int64_t n, int32_t every);

/* Replay: decisions logged by another implementation for attempts that
 * fall inside the 1e-9 band.  Metropolis keys (walker, sweep, attempt);
 * exchange keys (step, stage, lower slot).  The oracle adopts a logged
 * decision only where its own |x| <= 1e-9. */
void orc_pt_set_replay(orc_pt *p, int64_t nmet, const int64_t *met_w, const int64_t *met_n,
                       const int64_t *met_t, const int8_t *met_dec, int64_t nex,
                       const int64_t *ex_m, const int64_t *ex_g, const int64_t *ex_k,
                       const int8_t *ex_dec);

/* Getters.  Arrays are caller-allocated. */
void orc_pt_get_spins(const orc_pt *p, uint8_t *out);  /* [R][L] by walker, 1..q */
void orc_pt_get_perm(const orc_pt *p, int32_t *out);   /* [R] slot -> walker */
void orc_pt_get_energy(const orc_pt *p, double *out);  /* [R] tracked E by walker */
void orc_pt_get_stats(const orc_pt *p, double *sum6 /*[6][R]*/, int64_t *flip_att,
                      int64_t *flip_acc, int64_t *xchg_att, int64_t *xchg_acc, int64_t *counts3);
int64_t orc_pt_series_len(const orc_pt *p);
void orc_pt_get_series(const orc_pt *p, double *E /*[len][R]*/, double *M);
int64_t orc_pt_banded_count(const orc_pt *p);
/* Full O(L^2) energy of walker w (consistency check of the tracked value). */
double orc_pt_energy_full(const orc_pt *p, int32_t w);
void orc_pt_set_spins(orc_pt *p, const uint8_t *s);     /* [R][L], recomputes E and fields */

/* Separately written q = 2 path on +-1 spins: Metropolis at inverse
 * temperature beta_ising with the same draws as a Potts walker. */
int orc_ising_sweeps(int32_t L, const double *J, int8_t *sig, double beta_ising, uint64_t seed,
                     int32_t walker, int64_t sweep0, int64_t nsweeps, double *E_io);

#ifdef __cplusplus
}
#endif
#endif

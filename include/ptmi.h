/*
 * ptmi.h -- C ABI of the MI355X (gfx950) parallel-tempering library for the
 * 1D long-range q-state Potts ring.
 *
 * The method is that of Boer, "GPU-based simulation of the long-range Potts
 * model via parallel tempering" (Comput. Phys. Commun.):
 *   section 2, eqs. 1-3   spins s_i in 1..q, H = -sum J_ij delta(s_i, s_j),
 *                         each unordered pair {i, j} counted once;
 *   section 2, eqs. 4-7   periodic couplings J*(r) = sum_n |r + nL|^-(1+sigma),
 *                         evaluated with two Hurwitz zeta values;
 *   section 3, eq. 8      Metropolis single-spin flips, p = min(1, e^{-beta dE});
 *   section 3, eq. 9      replica exchange, p = min(1, e^{(E_i-E_j)(beta_i-beta_j)});
 *   section 4.2           exchange in two stages, pairs (i, i+1) with i even,
 *                         then with i odd (indices from 0);
 *   section 5.1, eqs. 10-12  M = (q Nmax/N - 1)/(q - 1), energy and Binder
 *                         cumulants (this library accumulates the moments).
 *
 * Random numbers come from Philox4x32-10 (Salmon et al., SC'11) with key
 * (lo32(seed), hi32(seed)).  Walker w, sweep n, attempt t (0 <= t < L) uses
 * counter (t, n, w, 0): site i = mulhi(o0, L), offset k = 1 + mulhi(o1, q-1),
 * new state b = ((a - 1 + k) mod q) + 1, u = ((o2 << 20 | o3 >> 12) + 1/2) 2^-52,
 * accepted iff beta dE + ln u < 0.  Exchange step m, stage g, lower slot k uses
 * counter (k, m, g, 1), u from (o0, o1), accepted iff ln u < (E_k - E_k+1)
 * (beta_k - beta_k+1).  Initial uniform spins: counter (j, 0, w, 2), s_j = 1 +
 * mulhi(o0, q).
 *
 * Ownership: the caller owns every host array it passes; arrays are read or
 * written during the call only (T is copied by pt_init).  All device memory
 * belongs to the context, either allocated by the library or carved from a
 * caller-provided device workspace (pt_options.workspace) that must stay
 * valid until pt_free.  Calls on one context are asynchronous on its stream
 * except where stated; calls on one context must not overlap.
 *
 * Errors: every function returns a pt_status; nothing aborts or throws
 * across the ABI.  pt_last_error() gives a thread-local message for the
 * last failing call of the calling thread.
 */
#ifndef PTMI_H
#define PTMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PT_OK = 0,
    PT_EINVAL = -1,   /* an argument is out of range or a pointer is NULL */
    PT_ENOMEM = -2,   /* device memory or workspace too small */
    PT_EDEVICE = -3,  /* a HIP call failed, or a kernel reported an error */
    PT_ESTATE = -4    /* call out of order, or on a freed/failed context */
} pt_status;

/* Precision of the field table.  F64: FP64 fields.  F32: FP32 fields with
 * FP64 rechecks of near-threshold attempts and refreshes when the rounding
 * drift reaches its cap.  I32: fields as exact int32 sums of couplings
 * quantised to 2^-k (k as large as keeps every field below 2^31): integer
 * updates are exact and order-free, so the table never drifts and is never
 * refreshed; near-threshold attempts (a constant band set by the quantisation)
 * are rechecked in FP64.  All three take every decision as the FP64 method
 * would (section 3, eq. 8); energies are tracked within a stated bound. */
enum { PT_PREC_F64 = 0, PT_PREC_F32 = 1, PT_PREC_I32 = 2 };
enum { PT_INIT_RANDOM = 0, PT_INIT_ORDERED = 1 };
/* Placement of a walker's field table during its sweeps: in LDS, in HBM
 * (couplings and spins in LDS), or no table at all (every energy change a
 * direct FP64 sum over the spins, the paper's own per-attempt scheme).  The
 * table keeps q - 1 rows of L entries per walker: a site's q fields sum to the
 * coupling sum, so the last row is formed from the others when read. */
enum { PT_PLACE_AUTO = 0, PT_PLACE_LDS = 1, PT_PLACE_HBM = 2, PT_PLACE_DIRECT = 3 };

/* Kernel limit on the number of Potts states. */
#define PT_QMAX 16
/* Half-width of the band in which two FP64 evaluations of beta dE + ln u may
 * legitimately disagree in sign; such decisions are logged as events. */
#define PT_BAND 1e-9

typedef struct {
    int32_t precision;      /* PT_PREC_F64, PT_PREC_F32 or PT_PREC_I32 (PT_PLACE_DIRECT
                               takes F64 or F32: it keeps no table) */
    int32_t init;           /* PT_INIT_RANDOM or PT_INIT_ORDERED (all spins 1) */
    int32_t placement;      /* PT_PLACE_*: where the field table lives during a sweep (AUTO:
                               LDS when it fits, else HBM; DIRECT: no table, direct sums) */
    int32_t threads;        /* threads per walker workgroup (multiple of 64, <= 256); 0 = auto
                               (single instance: 64 per 256 sites, at most 256; batch/server: 256);
                               512 (single instance, FP64 or int32 table in LDS, q <= 4,
                               256 <= L <= 1024): the overlapped sweep, the chain of each window
                               beside the previous window's flush in separate waves */
    int32_t refresh_every;  /* sweeps between O(L^2) recomputations of the fields; 0 = auto */
    int32_t series_capacity;/* sweeps of per-slot E and M to keep (0 = none) */
    int32_t event_capacity; /* entries of the banded-event log (0 = 4096) */
    int32_t max_sweeps_per_launch; /* 0 = auto */
    int32_t lds_budget;     /* batch/server: LDS bytes per walker workgroup (0 = all the device allows) */
    int32_t profile;        /* 1: keep per-walker phase counters (pt_get_phase_counters) */
    void *stream;           /* hipStream_t to run on, NULL = the null stream */
    void *workspace;        /* optional caller-owned device memory for all state */
    size_t workspace_bytes; /* its size; must be >= pt_workspace_size() */
} pt_options;

/* One near-threshold decision.  kind 0: Metropolis (a = walker, b = sweep,
 * c = attempt); kind 1: exchange (a = exchange step, b = stage, c = lower
 * slot).  x is the FP64 value of beta dE + ln u (kind 0) or ln u - Delta
 * (kind 1); decision is 1 for accepted. */
typedef struct {
    int64_t a, b, c;
    int32_t kind, decision;
    double x;
} pt_event;

/* Observables.  Every pointer may be NULL (skipped); arrays are caller-owned
 * host memory of the stated length.  "by slot" = by temperature index k,
 * T ascending as passed to pt_init. */
typedef struct {
    int32_t R, q, L;          /* out */
    int64_t sweeps;           /* sweeps done since pt_init */
    int64_t exchange_steps;   /* exchange steps done since pt_init */
    int64_t samples;          /* sweeps accumulated since the last pt_reset_stats */
    double *E, *M;            /* [R] current energy and magnetisation by slot */
    double *sumE, *sumE2, *sumE4, *sumM, *sumM2, *sumM4; /* [R] FP64 moments by slot */
    int64_t *flip_att, *flip_acc; /* [R] Metropolis attempts / accepts by slot */
    int64_t *xchg_att, *xchg_acc; /* [R-1] exchange attempts / accepts, pair (k, k+1) */
    int32_t *perm;            /* [R] slot -> walker */
    int64_t n_recheck;        /* FP64 direct rechecks of near-threshold attempts */
    int64_t n_banded;         /* decisions inside PT_BAND (Metropolis + exchange) */
    int64_t n_exact_energy;   /* exact O(L^2) energies computed for uncertain exchanges */
    int64_t n_refresh;        /* field recomputations */
    int64_t n_events_dropped; /* events beyond event_capacity */
} pt_obs;

typedef struct pt_ctx pt_ctx;

/* Fills *opt with defaults (FP64 table, random init, auto placement). */
void pt_default_options(pt_options *opt);

/* Device bytes pt_init needs for (L, q, R, opt); opt may be NULL. */
pt_status pt_workspace_size(int32_t L, int32_t q, int32_t R, const pt_options *opt, size_t *bytes);

/* Creates a run: computes J*(r) on the GPU (eq. 6, FP64), draws the initial
 * spins, builds the field table and the energies, sets perm = identity.
 *   2 <= L <= 65535; 2 <= q <= PT_QMAX; sigma > 0 (zeta(1+sigma) diverges at 0);
 *   T[R] > 0, finite, ascending (slot k has temperature T[k]); R >= 1.
 * On success *out owns the device state; the work is queued on the stream. */
pt_status pt_init(pt_ctx **out, int32_t L, int32_t q, double sigma, const double *T, int32_t R,
                  uint64_t seed, const pt_options *opt);

/* n sweeps of L Metropolis attempts per walker (eq. 8), observables
 * recorded per slot after each sweep, no exchange.  Asynchronous. */
pt_status pt_sweep(pt_ctx *ctx, int64_t n);

/* One exchange step (eq. 9): even stage then odd stage.  Asynchronous. */
pt_status pt_exchange(pt_ctx *ctx);

/* n sweeps with an exchange step after sweeps exchange_every, 2 exchange_every,
 * ... counted from the start of this call, in persistent cooperative launches
 * with a device-side grid barrier (no host round trip per sweep); the
 * schedule does not depend on how the sweeps are split into launches.
 * exchange_every = 0 behaves like pt_sweep.  Asynchronous. */
pt_status pt_run(pt_ctx *ctx, int64_t n, int32_t exchange_every);

/* Waits for queued work and copies observables to the host.  Synchronising. */
pt_status pt_observables(pt_ctx *ctx, pt_obs *out);

/* Spins by walker [R][L], values 1..q, and perm [R] (either may be NULL).
 * Synchronising. */
pt_status pt_get_spins(pt_ctx *ctx, uint8_t *spins_out, int32_t *perm_out);

/* J*(r), r = 0..L-1, as computed on the GPU (FP64).  Synchronising. */
pt_status pt_get_jstar(pt_ctx *ctx, double *out);

/* Per-sweep E and M by slot, [n][R] each, for the first min(recorded,
 * capacity) sweeps since pt_init; *n_out receives the row count. */
pt_status pt_get_series(pt_ctx *ctx, double *E, double *M, int64_t cap_rows, int64_t *n_out);

/* Logged near-threshold events (up to cap); *n_out receives the count stored. */
pt_status pt_get_events(pt_ctx *ctx, pt_event *out, int64_t cap, int64_t *n_out);

/* The launch plan chosen at pt_init: placement (PT_PLACE_LDS, _HBM or
 * _DIRECT), threads per walker workgroup and LDS bytes per workgroup of the
 * persistent sweep launch.  Any pointer may be NULL.  Host only. */
pt_status pt_get_plan(pt_ctx *ctx, int32_t *placement, int32_t *threads, int32_t *lds_bytes);

/* Phase counters of each walker, kept when pt_options.profile was set at
 * pt_init: shader-clock cycles (s_memtime) its workgroup spent in each phase,
 * summed over every launch since pt_init, and event counts.  out is caller
 * host memory of R * PT_PHASE_N uint64, by walker.  Synchronising.
 * PT_ESTATE if profiling is off. */
enum {
    PT_PHASE_DRAW = 0,      /* Philox draws of the attempts, staged in LDS            */
    PT_PHASE_CHAIN = 1,     /* Metropolis decisions (eq. 8) through the windows        */
    PT_PHASE_FLUSH = 2,     /* accepted flips applied to the field table               */
    PT_PHASE_RECORD = 3,    /* end-of-sweep energy sums, observables, refreshes        */
    PT_PHASE_EXCHANGE = 4,  /* device barrier and exchange step (eq. 9)                */
    PT_PHASE_TOTAL = 5,     /* the walker's whole loop                                 */
    PT_PHASE_WINDOWS = 6,   /* count: windows of 64 attempts                           */
    PT_PHASE_FLUSHES = 7,   /* count: windows with flips to apply                      */
    PT_PHASE_FLIPS = 8,     /* count: accepted flips                                   */
    PT_PHASE_ITERS = 9,     /* count: guess-and-check iterations of the chain          */
    /* the chain's cycles by step of its iterations (single instances; part of CHAIN): */
    PT_PHASE_CHAIN_GUESS = 10,    /* sure accepts guessed, same-site cut, compaction   */
    PT_PHASE_CHAIN_CORRECT = 11,  /* guessed flips applied to the later lanes' dE      */
    PT_PHASE_CHAIN_CHECK = 12,    /* re-decisions, commits, counters                   */
    PT_PHASE_CHAIN_RESOLVE = 13,  /* first differing lane decided, later lanes rebuilt */
    PT_PHASE_CHAIN_REDO = 14,     /* lanes whose site changed: dE re-derived           */
    PT_PHASE_CHAIN_SYNC = 15,     /* workgroup barrier closing an iteration            */
    PT_PHASE_N = 16
};
pt_status pt_get_phase_counters(pt_ctx *ctx, uint64_t *out);

/* Zeroes the moment and acceptance accumulators (e.g. after burn-in). */
pt_status pt_reset_stats(pt_ctx *ctx);

/* Blocks until all queued work of the context has finished; reports device
 * errors raised by kernels (e.g. a grid-barrier time-out). */
pt_status pt_synchronize(pt_ctx *ctx);

/* Checkpoint: the complete state is (spins, perm, sweep and exchange
 * counters, accumulators, seed, parameters); fields are rebuilt on load.
 * pt_save with buf == NULL returns the needed size in *len.  pt_load checks a
 * buffer on the host before any device call (sizes, every spin below q, perm
 * a permutation) and returns PT_EINVAL for a corrupt one. */
pt_status pt_save(pt_ctx *ctx, void *buf, size_t *len);
pt_status pt_load(pt_ctx **out, const void *buf, size_t len, const pt_options *opt);

/* Releases device memory (not a caller workspace) and the context. */
pt_status pt_free(pt_ctx *ctx);

/* Thread-local message of the last failure on this thread ("" if none). */
const char *pt_last_error(void);

/* ------------------------------------------------------------------------ */
/* Without allocation.  For callers that cannot allocate device memory: code */
/* running under stream capture, tight serving loops, harnesses that forbid */
/* hipMalloc.  pt_run_static does what pt_init, pt_run(n, exchange_every),  */
/* pt_observables and pt_get_spins do together, with the same kernels and   */
/* the same results, but keeps the whole device state in one static device */
/* buffer of PT_STATIC_SCRATCH_BYTES per GPU, which the library owns.  Each */
/* GPU the library runs on holds that buffer from the library's first use of */
/* it on that GPU until the process ends.  No hipMalloc, hipFree or other    */
/* allocating routine is called, on the device or the host.                 */
/* ------------------------------------------------------------------------ */
#define PT_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* Arguments as pt_init (L, q, sigma, T[R] ascending, seed, opt: precision,
 * init, placement, threads, event_capacity, max_sweeps_per_launch and stream
 * are honoured; series_capacity and profile are ignored; opt->workspace must
 * be NULL), then n sweeps with an exchange step after every exchange_every-th
 * (0: none), as pt_run.  Outputs, each optional (NULL = skipped), caller-owned
 * host memory: *out as pt_observables, spins_out[R * L] and perm_out[R] as
 * pt_get_spins.  Synchronises the stream before it returns.
 * PT_EINVAL if the state (the pt_init workspace of these sizes plus 16 R bytes)
 * exceeds PT_STATIC_SCRATCH_BYTES, as well as for any argument pt_init or
 * pt_run would refuse.  Every call on one GPU uses that GPU's one buffer and
 * leaves its state there: host threads calling on the same GPU are serialised
 * by the library, and no other work may touch the buffer, so calls whose device
 * work would overlap on one GPU (e.g. from another process sharing its memory)
 * race. */
pt_status pt_run_static(int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed, int64_t n,
                        int32_t exchange_every, const pt_options *opt, pt_obs *out, uint8_t *spins_out,
                        int32_t *perm_out);

/* ------------------------------------------------------------------------ */
/* Batches: many independent instances of uneven size in one persistent    */
/* launch.  Workgroups take walkers job by job from a ticket counter, so a */
/* job's walkers always meet at its exchange barrier; each job runs `sweeps`*/
/* sweeps with an exchange step after every `exchange_every`-th.  Results  */
/* per job equal those of the same job run alone (same streams).           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t L, q;            /* as pt_init */
    double sigma;
    const double *T;         /* [R] ascending; copied at creation */
    int32_t R;
    uint64_t seed;
    int64_t sweeps;          /* >= 0 */
    int32_t exchange_every;  /* >= 1 */
    int32_t init;            /* PT_INIT_RANDOM or PT_INIT_ORDERED */
} pt_job_desc;

typedef struct pt_batch pt_batch;

/* Device bytes for a batch (all jobs' state plus the job table). */
pt_status pt_batch_workspace_size(const pt_job_desc *jobs, int32_t njobs, const pt_options *opt, size_t *bytes);
/* Validates and lays out the jobs; opt->threads and opt->lds_budget pick the
 * walker workgroup shape (0 = auto).  Nothing runs yet. */
pt_status pt_batch_create(pt_batch **out, const pt_job_desc *jobs, int32_t njobs, const pt_options *opt);
/* One launch that sets up and runs every job to completion.  Asynchronous. */
pt_status pt_batch_run(pt_batch *b);
/* Observables and spins of job `job` after pt_batch_run (synchronising). */
pt_status pt_batch_observables(pt_batch *b, int32_t job, pt_obs *out);
pt_status pt_batch_get_spins(pt_batch *b, int32_t job, uint8_t *spins_out, int32_t *perm_out);
/* Workgroups used by the launch and threads per workgroup (for reporting). */
pt_status pt_batch_shape(pt_batch *b, int32_t *workgroups, int32_t *threads, int32_t *lds_bytes);
/* Placement of job `job`'s field table (PT_PLACE_LDS, _HBM or _DIRECT), and,
 * after pt_batch_run (synchronising), the device wall clock in seconds when
 * the job's set-up began and when its last walker finished (a clock common to
 * every job of the launch).  Any pointer may be NULL. */
pt_status pt_batch_job_stats(pt_batch *b, int32_t job, int32_t *placement, double *start_s, double *end_s);
pt_status pt_batch_free(pt_batch *b);

/* ------------------------------------------------------------------------ */
/* Serving: a persistent launch that keeps taking jobs while it runs.      */
/* Submitted jobs wait in a host queue, in order, until their state fits in */
/* the device arena (admission by device memory) and the walkers admitted   */
/* and not yet finished stay within twice the resident workgroups; they are */
/* then published to the running kernel, and their results are copied back */
/* when their last walker ends.  A host thread does the admission,          */
/* publication and completion polling.                                      */
/* ------------------------------------------------------------------------ */
typedef struct pt_server pt_server;

/* Device bytes a server needs for an arena of arena_bytes and max_jobs
 * submissions: the size of a caller workspace (opt->workspace) for it. */
pt_status pt_server_workspace_size(size_t arena_bytes, int32_t max_jobs, size_t *bytes);
/* arena_bytes of device memory for job state (opt->workspace may supply it);
 * max_jobs bounds the number of submissions over the server's life.  The
 * server's kernel stays resident until pt_server_stop: a device-wide
 * synchronisation (hipDeviceSynchronize) issued by the caller while the server
 * runs never returns. */
pt_status pt_server_start(pt_server **out, size_t arena_bytes, int32_t max_jobs, const pt_options *opt);
/* Queues a job (T copied); *id_out receives its id.  Thread-safe. */
pt_status pt_server_submit(pt_server *s, const pt_job_desc *job, int64_t *id_out);
/* *done_out = 1 when job id has finished; then fills *out if non-NULL. */
pt_status pt_server_poll(pt_server *s, int64_t id, int32_t *done_out, pt_obs *out);
/* Blocks until job id has finished (or timeout_s elapses: PT_ESTATE). */
pt_status pt_server_wait(pt_server *s, int64_t id, double timeout_s, pt_obs *out);
/* Cancels job id if it still waits in the host queue (PT_OK; poll then
 * reports it ended and wait/poll/get_spins return PT_ESTATE for it); a job
 * already admitted runs to its end (PT_ESTATE).  Thread-safe. */
pt_status pt_server_cancel(pt_server *s, int64_t id);
/* Host times of job id (seconds on a monotonic clock): submitted, admitted
 * (published to the device), finished (results copied back). */
pt_status pt_server_times(pt_server *s, int64_t id, double *submitted, double *admitted, double *finished);
/* Spins [R][L] (1..q) and perm [R] of a finished job. */
pt_status pt_server_get_spins(pt_server *s, int64_t id, uint8_t *spins_out, int32_t *perm_out);
/* Drains every submitted job, stops the persistent launch, frees the server. */
pt_status pt_server_stop(pt_server *s);

#ifdef __cplusplus
}
#endif
#endif /* PTMI_H */

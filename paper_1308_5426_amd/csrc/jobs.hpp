// jobs.hpp -- one persistent launch for many instances ("jobs") of uneven size.
//
// Each workgroup repeatedly claims a ticket.  Tickets are numbered job by job
// (job j owns tickets wbase_j .. wbase_j + R_j - 1, one per walker), so at any
// time at most one job is partly claimed: every job with a lower ticket range
// is fully claimed and runs to completion, freeing workgroups that then claim
// the rest.  With at least max_j R_j workgroups resident, the per-job device
// barriers therefore always fill and the launch cannot deadlock.
//
// A claimed walker sets up its own state: walker 0 clears the job's counters,
// computes its couplings (eq. 6) and publishes them; every walker draws its
// initial spins, builds its field table and runs the job's sweeps with the
// exchange after each (the same code as a single instance).  The last walker
// to finish marks the job done; a walker that gave up (barrier time-out) still
// counts, with an error bit, so a failed job ends instead of hanging.
//
// A static batch has a fixed job count and its table in device memory,
// written before the launch.  A server keeps publishing jobs while the launch
// runs: its job table and ladders live in coherent (fine-grained) pinned host
// memory, written by the host before it raises the published count (such
// memory is coherent with a running kernel, unlike host copies into device
// memory during a launch, or default pinned memory).  Nothing the
// device reads of a job comes from such a copy: the ready/finished words are one
// pair per slot, never reused and cleared before the launch, and the counters
// in the job's (reused) arena block are cleared by the device itself.
#pragma once
#include "sweep.hpp"

namespace ptmi {

// Kernel variant of a job: placement of its field table (kPl*, bits 0-1), rows
// held in registers by the flush for the q - 1 stored rows (bits 2-4: 0 none,
// 1 four, 2 eight, 3 six, 4 two) and FP64 couplings in LDS (bit 5).
constexpr int32_t kVarQtShift = 2, kVarQtMask = 7, kVarJ64Lds = 32;
__host__ __device__ inline int32_t job_variant(int place, int q, bool j64_in_lds)
{
    const int32_t qt = q <= 3 ? 4 : (q <= 4 ? 1 : (q <= 6 ? 3 : (q <= 8 ? 2 : 0)));
    return static_cast<int32_t>(place) | (qt << kVarQtShift) | (j64_in_lds ? kVarJ64Lds : 0);
}

// Per-job device words: [0] couplings ready, [1] walkers finished, [2] the
// device wall clock when walker 0 began the set-up, [3] when the last walker
// finished (wall_clock64 ticks).
constexpr int kJcWords = 4;

struct alignas(256) JobSlot {
    Inst inst;
    LdsPlan plan;      // carve of this job inside the launch's LDS budget
    const double *T;   // [R] ascending temperatures (device or pinned host memory)
    unsigned long long *jc;  // [kJcWords] couplings ready, walkers finished, start and end clocks (device
                             // memory, zero at launch)
    double sigma;
    int64_t sweeps;
    int32_t xevery;
    int32_t init;
    int32_t wbase;     // first ticket of the job
    int32_t variant;   // kVar* bits
};

struct JobControl {
    unsigned ticket;   // next ticket (device memory)
    unsigned pad[63];
};

__device__ __forceinline__ int32_t load_published(const int32_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Set-up and sweeps of walker w of job S, then the job's completion count.
template <typename F, int QT, int PL, bool J64L>
__device__ __forceinline__ void run_job_walker(const JobSlot &S, int w, unsigned char *lds, int32_t *done_flag, int32_t *sflag)
{
    // the slot may sit in host memory (serving): read it once
    Inst P = S.inst;
    const LdsPlan plan = S.plan;
    unsigned long long *const jc = S.jc;
    const int tid = threadIdx.x, L = P.L, R = P.R;
    if (w == 0) {
        if (tid == 0) jc[2] = wall_clock64();
        // the job's counters (the arena block may have held an earlier job),
        // couplings, error bounds, ladder and zeroed accumulators
        for (int k = tid; k < kCtrN; k += blockDim.x) P.ctr[k] = 0ull;
        for (int r = tid; r <= L / 2; r += blockDim.x)
            jstar_entry(L, S.sigma, r, const_cast<double *>(P.J64), const_cast<float *>(P.J32));
        for (int k = tid; k < R; k += blockDim.x) {
            const_cast<double *>(P.beta)[k] = 1.0 / S.T[k];
            P.perm[k] = k;
            P.slot_of[k] = k;
            P.fatt[k] = 0; P.facc[k] = 0; P.xatt[k] = 0; P.xacc[k] = 0;
            for (int a = 0; a < 6; ++a) P.acc6[a * R + k] = 0.0;
        }
        __syncthreads();
        // the same sums, in the same order, as a single instance's k_setup
        setup_couplings(P, table_prec<F>());
        release_all_agent();  // every thread's part of the set-up, before the ready flag
        if (tid == 0) __hip_atomic_store(&jc[0], 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) {
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&jc[0], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0ull) {
            __builtin_amdgcn_s_sleep(8);
            if (wall_clock64() - t0 > kBarrierTicks) {
                ok = 0;
                break;
            }
        }
        sflag[0] = ok;
    }
    acquire_all_agent();  // walker 0's set-up, in every thread
    bool ok = sflag[0] != 0;
    if (ok) {
        P.bound_init = __hip_atomic_load(&P.bnd->init, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.bound_unit = __hip_atomic_load(&P.bnd->unit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.nupd_max = __hip_atomic_load(&P.bnd->nupd_max, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.bound_flipE = __hip_atomic_load(&P.bnd->flipE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.ebound = __hip_atomic_load(&P.bnd->ebound, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.qscale = __hip_atomic_load(&P.bnd->qscale, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.hsum = __hip_atomic_load(&P.bnd->hsum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.bound_rows = __hip_atomic_load(&P.bnd->rows, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        P.bound_impl = __hip_atomic_load(&P.bnd->impl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int j = tid; j < L; j += blockDim.x)
            P.spins[static_cast<size_t>(w) * L + j] = initial_spin(P, w, j, S.init != 0);
        __syncthreads();
        Walker<F> W = carve<F, PL, J64L>(lds, plan, P, w);
        load_walker<F>(P, W, plan, w);
        const double E = refresh_fields<F>(P, W);
        __syncthreads();
        store_walker<F>(P, W, plan, w);
        if (tid == 0) {
            P.E[w] = E;
            P.Eerr[w] = P.ebound;
            P.nupd[w] = 0;
            int nmax = 0;
            for (int k = 0; k < P.q; ++k) nmax = max(nmax, W.cnt[k]);
            P.Mw[w] = (static_cast<double>(P.q) * nmax / L - 1.0) / (P.q - 1);
        }
        __syncthreads();
        ok = run_walker<F, QT, PL, J64L>(P, plan, lds, w, 0, static_cast<int32_t>(S.sweeps), S.xevery, 0, 0, true);
    }
    // every thread's final writes of this walker visible to the host (which
    // copies the job's results once its last walker is counted)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __syncthreads();
    if (tid == 0) {
        if (!ok) atomicOr(&P.ctr[kCtrError], kErrBarrierTimeout);
        __threadfence_system();
        const unsigned long long d = __hip_atomic_fetch_add(&jc[1], 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d == static_cast<unsigned long long>(R) - 1ull) {
            jc[3] = wall_clock64();
            if (done_flag) {
                __threadfence_system();
                __hip_atomic_store(done_flag, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
        }
    }
    __syncthreads();
}

template <typename F, int PL, bool J64L>
__device__ __forceinline__ void dispatch_qt(const JobSlot &S, int w, unsigned char *lds, int32_t *done_flag, int32_t *sflag)
{
    if constexpr (PL == kPlDirect) {
        run_job_walker<F, 0, PL, J64L>(S, w, lds, done_flag, sflag);
    } else {
        switch ((S.variant >> kVarQtShift) & kVarQtMask) {
        case 4: run_job_walker<F, 2, PL, J64L>(S, w, lds, done_flag, sflag); break;
        case 1: run_job_walker<F, 4, PL, J64L>(S, w, lds, done_flag, sflag); break;
        case 2: run_job_walker<F, 8, PL, J64L>(S, w, lds, done_flag, sflag); break;
        case 3: run_job_walker<F, 6, PL, J64L>(S, w, lds, done_flag, sflag); break;
        default: run_job_walker<F, 0, PL, J64L>(S, w, lds, done_flag, sflag); break;
        }
    }
}

template <typename F, int PL>
__device__ __forceinline__ void dispatch_j64(const JobSlot &S, int w, unsigned char *lds, int32_t *done_flag, int32_t *sflag)
{
    if constexpr (table_prec<F>() == kPrecF64)  // FP64 couplings are the table's own, always in LDS
        dispatch_qt<F, PL, true>(S, w, lds, done_flag, sflag);
    else if constexpr (table_prec<F>() == kPrecI32)  // never in LDS
        dispatch_qt<F, PL, false>(S, w, lds, done_flag, sflag);
    else if (S.variant & kVarJ64Lds)
        dispatch_qt<F, PL, true>(S, w, lds, done_flag, sflag);
    else
        dispatch_qt<F, PL, false>(S, w, lds, done_flag, sflag);
}

template <typename F>
__device__ __forceinline__ void dispatch_job_walker(const JobSlot &S, int w, unsigned char *lds, int32_t *done_flag, int32_t *sflag)
{
    switch (S.variant & 3) {
    case kPlLds: dispatch_j64<F, kPlLds>(S, w, lds, done_flag, sflag); break;
    case kPlHbm: dispatch_j64<F, kPlHbm>(S, w, lds, done_flag, sflag); break;
    default:  // batches plan LDS or HBM tables; direct sums are no int form
        if constexpr (table_prec<F>() != kPrecI32) dispatch_j64<F, kPlDirect>(S, w, lds, done_flag, sflag);
        break;
    }
}

// nstatic >= 0: a batch of nstatic jobs (slots in device memory); the launch
// ends when every ticket is taken.  nstatic < 0: serving; the slots are in
// pinned host memory, *published (host memory) counts the valid ones, *stop
// (host memory) ends the launch once no published ticket is left.
template <typename F>
__global__ __launch_bounds__(kMaxJobThreads) void k_jobs(const JobSlot *slots, int32_t nstatic,
                                                           const int32_t *published, const int32_t *stop,
                                                           JobControl *ctl, int32_t *done_flags)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ int32_t sh[4];
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0) {
            const int t = static_cast<int>(atomicAdd(&ctl->ticket, 1u));
            int found = -1;
            for (;;) {
                const int npub = nstatic >= 0 ? nstatic : load_published(published);
                // the job whose ticket range holds t: last slot with wbase <= t
                int lo = 0, hi = npub - 1;
                while (lo <= hi) {
                    const int mid = (lo + hi) >> 1;
                    if (slots[mid].wbase <= t) {
                        found = mid;
                        lo = mid + 1;
                    } else {
                        hi = mid - 1;
                    }
                }
                if (found >= 0 && t >= slots[found].wbase + slots[found].inst.R) found = -1;
                if (found >= 0 || nstatic >= 0) break;
                if (__hip_atomic_load(stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM) != 0 &&
                    load_published(published) == npub)
                    break;
                __builtin_amdgcn_s_sleep(64);
            }
            sh[0] = found;
            sh[1] = found >= 0 ? t - slots[found].wbase : 0;
        }
        __syncthreads();
        const int j = sh[0], w = sh[1];
        if (j < 0) return;
        dispatch_job_walker<F>(slots[j], w, lds, done_flags ? done_flags + j : nullptr, sh + 2);
        __syncthreads();
    }
}

}  // namespace ptmi

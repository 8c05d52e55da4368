// sweep.hpp -- gfx950 kernels of the parallel-tempering hot path:
//   k_init_spins   initial spins from the walker's Philox stream
//   k_refresh<F>   O(L^2) field table h[k][j] = sum_{i != j} J*(|i-j|) delta(s_i, k),
//                  FP64 accumulation, stored as F; exact energy and state counts
//   k_sweep<F>     Metropolis sweeps (eq. 8) with O(1) dE from the LDS field
//                  table and an O(L) workgroup-parallel update per accepted flip;
//                  optionally persistent with a device-side grid barrier and the
//                  exchange step (eq. 9) run by the last workgroup to arrive
//   k_exchange     the two-stage exchange step (section 4.2) as its own launch
//
// One workgroup owns one walker (replica).  The attempts of a sweep are taken
// in windows of 64 consecutive attempts, lane = attempt.  Wave 0 runs the
// Markov chain through the window: every lane holds the local fields of its
// site for all q states in registers; the first lane that is accepted (or
// needs an FP64 recheck) is applied, every earlier lane was a rejection and
// changed nothing, and the later lanes correct their fields by the coupling
// to the flipped site.  This keeps the sequential semantics of the chain
// exactly while each accepted flip costs one LDS gather instead of an O(L)
// table update.  At the end of the window the whole workgroup applies the
// window's flips to the LDS table in one pass (each thread owns a set of
// sites and applies the flips in order, so no barrier is needed between
// them).
#pragma once
#include <type_traits>

#include "device_common.hpp"
#include "state.hpp"

namespace ptmi {

// LDS carve (byte offsets), computed on the host by lds_plan().
struct LdsPlan {
    int32_t J, h, J64, masks, sp, cnt, red, misc, xch, draw, dlnu, pend, cs, total;
    int32_t j64_in_lds;   // 1: FP64 couplings resident in LDS
    int32_t h_in_lds;     // 1: field table in LDS; 0: in HBM, or no table (place)
    int32_t place;        // kPlLds, kPlHbm or kPlDirect
    int32_t chunk;        // attempts whose draws are staged in LDS at a time (multiple of 64)
    int32_t jlen;         // entries of the coupling row J: L, or L + flush span when doubled
    int32_t sfirst;       // [waves][L] u32 first-guessed-flip tables, or -1 when they do not fit
    int32_t xpart;        // [2][waves][64] FP64 partial corrections exchanged between waves
    int32_t ctab;         // [64][4] flush coefficients (table precision) by flip kind
    int32_t ovl;          // 1: overlapped sweep (chain in the first half of the waves, flush in the second)
};

// Where a walker's field table lives during its sweeps (values of
// PT_PLACE_*): in LDS (with a doubled coupling row), in HBM (couplings and
// spins in LDS, the table's rows read and written through the caches), or no
// table at all (every energy change a direct FP64 sum over the spins).
enum : int { kPlLds = 1, kPlHbm = 2, kPlDirect = 3 };

// Flush geometry: in each pass every wave owns kFlushM blocks of 64
// consecutive sites; thread (wave v, lane l) holds sites
// jb + v * 64 * kFlushM + 64 m + l, m < kFlushM.
constexpr int kFlushM = 4;
// Flips whose couplings are gathered together before they are applied.
constexpr int kFlipBatch = 4;

// Scalars of the walker's chain, kept by wave 0 and published through LDS.
struct ChainState {
    double E, Eerr;
    int64_t nupd, nacc;
    int32_t np[2];
    int32_t pad[2];
};

// Margin for the FP64 evaluation of beta dE + ln u beyond the table bound
// (FP64 rounding of the products and of the library logarithm).
constexpr double kEvalMargin = 1e-12;
// Workgroup size limit of the walker kernels: one wave per SIMD, so every wave
// may use the whole register file.
constexpr int kMaxSweepThreads = 256;
constexpr int kMaxJobThreads = 256;
// Grid barrier time-out, in wall-clock ticks (100 MHz on gfx9): 20 s.
constexpr uint64_t kBarrierTicks = 2000000000ull;

template <typename F>
struct Walker {
    F *J;               // [L] couplings in the table's precision
    F *h;               // [q-1][L] field table (row q-1 implicit: the coupling sum minus the others)
    const double *J64;  // [L] FP64 couplings (LDS or HBM)
    uint8_t *sp;        // [L] spins 0..q-1
    int32_t *cnt;       // [kQMax]
    uint64_t *masks;    // [q][ceil(L/64)] sites per state, for the refresh
    double *red;        // [16] reduction scratch
    int32_t *misc;      // [8]
    uint32_t *draw;     // [chunk] site | offset << 16
    double *dlnu;       // [chunk] ln u
    uint32_t *pend;     // [64] flip words of the flips accepted in the current window
    uint32_t *sfirst;   // [waves][L] per site: first lane of the current guess flipping it (64: none), or null
    double *xpart;      // [2][waves][64] partial corrections of the split passes
    F *ctab;            // [64][4] row coefficients of a flip of kind old + 16 new (states < 4)
    ChainState *cs;
    uint32_t *gbar;     // [2] arrivals and generation of the chain waves' LDS barrier (overlapped sweep)
    unsigned long long *err;  // the instance's error bits (bounded waits)
    int32_t chunk;
};

// PL / J64L: where the field table is (kPl*) / whether the FP64 couplings
// are in LDS.  They are compile-time choices so that every access compiles to
// ds_* (LDS) or global_* (HBM) instructions rather than flat ones.
template <typename F, int PL, bool J64L>
__device__ __forceinline__ Walker<F> carve(unsigned char *lds, const LdsPlan &p, const Inst &P, int w)
{
    Walker<F> W;
    W.J = reinterpret_cast<F *>(lds + p.J);
    if constexpr (PL == kPlLds)
        W.h = reinterpret_cast<F *>(lds + p.h);
    else
        W.h = static_cast<F *>(P.h) + static_cast<size_t>(w) * (P.q - 1) * P.L;
    if constexpr (J64L)
        W.J64 = reinterpret_cast<const double *>(lds + p.J64);
    else
        W.J64 = P.J64;
    W.sp = lds + p.sp;
    W.cnt = reinterpret_cast<int32_t *>(lds + p.cnt);
    W.masks = reinterpret_cast<uint64_t *>(lds + p.masks);
    W.red = reinterpret_cast<double *>(lds + p.red);
    W.misc = reinterpret_cast<int32_t *>(lds + p.misc);
    W.draw = reinterpret_cast<uint32_t *>(lds + p.draw);
    W.dlnu = reinterpret_cast<double *>(lds + p.dlnu);
    W.pend = reinterpret_cast<uint32_t *>(lds + p.pend);
    W.cs = reinterpret_cast<ChainState *>(lds + p.cs);
    W.sfirst = p.sfirst >= 0 ? reinterpret_cast<uint32_t *>(lds + p.sfirst) : nullptr;
    W.xpart = reinterpret_cast<double *>(lds + p.xpart);
    W.ctab = reinterpret_cast<F *>(lds + p.ctab);
    W.gbar = reinterpret_cast<uint32_t *>(W.misc + 4);
    W.err = P.ctr + kCtrError;
    W.chunk = p.chunk;
    return W;
}

template <typename F>
__device__ __forceinline__ const F *coupling_src(const Inst &P);
template <>
__device__ __forceinline__ const float *coupling_src<float>(const Inst &P) { return P.J32; }
template <>
__device__ __forceinline__ const double *coupling_src<double>(const Inst &P) { return P.J64; }
template <>
__device__ __forceinline__ const int32_t *coupling_src<int32_t>(const Inst &P) { return P.Jq; }

template <typename F>
constexpr int table_prec()
{
    return sizeof(F) == sizeof(double) ? kPrecF64 : (__is_same(F, float) ? kPrecF32 : kPrecI32);
}

__device__ __forceinline__ void log_event(const Inst &P, int kind, int64_t a, int64_t b, int64_t c,
                                          int dec, double x)
{
    const unsigned long long at = atomicAdd(&P.ctr[kCtrEvents], 1ull);
    if (at < static_cast<unsigned long long>(P.ev_cap)) {
        Event e;
        e.a = a; e.b = b; e.c = c; e.kind = kind; e.decision = dec; e.x = x;
        P.events[at] = e;
    }
}

// ---------------------------------------------------------------------------
// Initial spins (counter (j, 0, w, 2)) or the ordered state.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint8_t initial_spin(const Inst &P, int w, int j, bool ordered)
{
    if (ordered) return 0;
    const uint4 o = philox10(make_uint4(static_cast<uint32_t>(j), 0u, static_cast<uint32_t>(w), 2u), P.key0, P.key1);
    return static_cast<uint8_t>(__umulhi(o.x, static_cast<uint32_t>(P.q)));
}

static __global__ void k_init_spins(Inst P, int32_t ordered)
{
    const int64_t total = static_cast<int64_t>(P.R) * P.L;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int w = static_cast<int>(e / P.L), j = static_cast<int>(e % P.L);
        P.spins[e] = initial_spin(P, w, j, ordered != 0);
    }
}

// ---------------------------------------------------------------------------
// Walker state HBM <-> LDS.
// ---------------------------------------------------------------------------
// Change of the field of state c under a flip ap -> bp, in units of the
// coupling: -1 if c was the old state, +1 if c is the new one, else 0.  Applied
// as fma(coef, J, h), which rounds exactly as h - J or h + J (or leaves h).
template <typename F>
__device__ __forceinline__ F flip_coef(int c, int ap, int bp)
{
    // +1 for the new state, -1 for the old one; 0 otherwise, and for ap == bp (no flip)
    return c == bp ? (c == ap ? F(0) : F(1)) : (c == ap ? F(-1) : F(0));
}

template <typename F>
__device__ __forceinline__ void load_walker(const Inst &P, Walker<F> &W, const LdsPlan &plan, int w)
{
    const int L = P.L, q = P.q;
    const F *Jsrc = coupling_src<F>(P);
    const F *hsrc = static_cast<const F *>(P.h) + static_cast<size_t>(w) * (q - 1) * L;
    const uint8_t *ssrc = P.spins + static_cast<size_t>(w) * L;
    double *J64l = plan.j64_in_lds && sizeof(F) != sizeof(double) ? const_cast<double *>(W.J64) : nullptr;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        W.sp[j] = ssrc[j];
        if (J64l) J64l[j] = P.J64[j];
    }
    const int chain_waves = static_cast<int>(blockDim.x / kWave) / (plan.ovl ? 2 : 1);
    if (W.sfirst)
        for (int k = threadIdx.x; k < chain_waves * L; k += blockDim.x) W.sfirst[k] = kWave;
    if (threadIdx.x < 2) W.gbar[threadIdx.x] = 0u;
    // coefficient of row c under a flip ap -> bp, kind ap + 16 bp (kind 0: no flip)
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int k = e >> 2, c = e & 3;
        W.ctab[e] = flip_coef<F>(c, k & 15, k >> 4);
    }
    // J[k] = J*(k mod L): with a doubled row, J*(|j - i|) = J[j - i + L] needs no wrap
    for (int k = threadIdx.x; k < plan.jlen; k += blockDim.x) W.J[k] = Jsrc[k % L];
    if (plan.h_in_lds)
        for (int e = threadIdx.x; e < (q - 1) * L; e += blockDim.x) W.h[e] = hsrc[e];
    if (threadIdx.x < kQMax) W.cnt[threadIdx.x] = P.counts[w * kQMax + threadIdx.x];
}

template <typename F>
__device__ __forceinline__ void store_walker(const Inst &P, const Walker<F> &W, const LdsPlan &plan, int w)
{
    const int L = P.L, q = P.q;
    F *hdst = static_cast<F *>(P.h) + static_cast<size_t>(w) * (q - 1) * L;
    uint8_t *sdst = P.spins + static_cast<size_t>(w) * L;
    for (int j = threadIdx.x; j < L; j += blockDim.x) sdst[j] = W.sp[j];
    if (plan.h_in_lds)
        for (int e = threadIdx.x; e < (q - 1) * L; e += blockDim.x) hdst[e] = W.h[e];
    if (threadIdx.x < kQMax) P.counts[w * kQMax + threadIdx.x] = W.cnt[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Field table from the spins, FP64 accumulation (exact for int tables).  For
// each state k a bitmask per 64-site block lists the sites in state k; every
// thread owns sites j and walks the set bits (wave-uniform, scalar), adding
// the coupling to j.  Rows 0 .. q-2 are stored (row q-1 is implicit).  The
// energy E = -1/2 sum_j h[s_j][j] (real units) is formed from the FP64 sums of
// every row.
// ---------------------------------------------------------------------------
template <typename F>
__device__ __forceinline__ double refresh_fields(const Inst &P, Walker<F> &W)
{
    const int L = P.L, q = P.q, tid = threadIdx.x, NT = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave, nw = NT / kWave;
    const int nblk = (L + kWave - 1) / kWave;
    __syncthreads();
    for (int blk = wv; blk < nblk; blk += nw) {
        const int j = blk * kWave + lane;
        const int s = j < L ? W.sp[j] : -1;
        for (int k = 0; k < q; ++k) {
            const uint64_t m = ballot(s == k);
            if (lane == 0) W.masks[k * nblk + blk] = m;
        }
    }
    __syncthreads();
    if (tid < kQMax) {
        int c = 0;
        if (tid < q)
            for (int blk = 0; blk < nblk; ++blk) c += __popcll(W.masks[tid * nblk + blk]);
        W.cnt[tid] = c;
    }
    double epart = 0.0;
    for (int j0 = 0; j0 < L; j0 += NT) {
        const int j = j0 + tid;
        const bool ok = j < L;
        const int jj = ok ? j : 0;
        const int sj = ok ? W.sp[j] : -1;
        for (int k = 0; k < q; ++k) {
            double acc = 0.0;
            for (int blk = 0; blk < nblk; ++blk) {
                const uint64_t mv = W.masks[k * nblk + blk];
                const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(mv));
                const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(mv >> 32));
                uint64_t m = (static_cast<uint64_t>(hi) << 32) | lo;
                while (m) {
                    const int bit = __builtin_ctzll(m);
                    m &= m - 1;
                    int d = jj - (blk * kWave + bit);
                    d += d < 0 ? L : 0;
                    // J*(0) = 0 removes the self term.  FP32 / int tables sum their
                    // own couplings (LDS), the FP64 table the FP64 ones.
                    if constexpr (table_prec<F>() == kPrecF64)
                        acc += W.J64[d];
                    else
                        acc += static_cast<double>(W.J[d]);
                }
            }
            if (ok) {
                if (k < q - 1) W.h[k * L + j] = static_cast<F>(acc);  // row q-1 is implicit
                if (k == sj) epart += acc;
            }
        }
    }
    return -0.5 * block_sum(epart, W.red) * P.qscale;
}

// Exact energy of walker w from its spins in HBM: E = -1/2 sum_j sum_{i != j}
// J*(|i-j|) delta(s_i, s_j).  O(L^2); used only for uncertain exchanges.
__device__ double exact_energy(const Inst &P, int w, double *red)
{
    const int L = P.L;
    const uint8_t *s = P.spins + static_cast<size_t>(w) * L;
    double part = 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const uint8_t sj = s[j];
        for (int i = 0; i < L; ++i) {
            if (s[i] != sj) continue;
            int d = j - i;
            d += d < 0 ? L : 0;
            part += P.J64[d];
        }
    }
    return -0.5 * block_sum(part, red);
}

// ---------------------------------------------------------------------------
// Exchange step m (eq. 9, section 4.2), run by one workgroup.  Energies are
// the tracked FP64 values with a rigorous error bound Eerr; a decision whose
// margin |ln u - Delta| is within |dbeta| (Eerr_a + Eerr_b) is resolved with
// exact O(L^2) energies.  Walkers keep their state; the slot labels move.
// ---------------------------------------------------------------------------
struct XScratch {
    int32_t *perm, *dec;
    double *E, *Eerr, *beta, *lnu;
};

__device__ __forceinline__ XScratch carve_x(unsigned char *base, int R)
{
    XScratch X;
    X.E = reinterpret_cast<double *>(base);
    X.Eerr = X.E + R;
    X.beta = X.Eerr + R;
    X.lnu = X.beta + R;
    X.perm = reinterpret_cast<int32_t *>(X.lnu + R);
    X.dec = X.perm + R;
    return X;
}

__device__ void exchange_step(const Inst &P, int64_t m, XScratch X, double *red)
{
    const int R = P.R, tid = threadIdx.x, NT = blockDim.x;
    __syncthreads();
    for (int k = tid; k < R; k += NT) {
        X.perm[k] = P.perm[k];
        X.E[k] = P.E[k];
        X.Eerr[k] = P.Eerr[k];
        X.beta[k] = P.beta[k];
    }
    __syncthreads();
    for (int g = 0; g < 2; ++g) {
        const int npair = (R - g) / 2;
        bool unsure = false;
        for (int p = tid; p < npair; p += NT) {
            const int k = g + 2 * p;
            const int wa = X.perm[k], wb = X.perm[k + 1];
            const double db = X.beta[k] - X.beta[k + 1];
            const uint4 o = philox10(make_uint4(static_cast<uint32_t>(k), static_cast<uint32_t>(m),
                                                static_cast<uint32_t>(g), 1u),
                                     P.key0, P.key1);
            const double lnu = log(open_unit(o.x, o.y));
            const double y = lnu - (X.E[wa] - X.E[wb]) * db;
            const double band = fabs(db) * (X.Eerr[wa] + X.Eerr[wb]);
            X.lnu[k] = lnu;
            X.dec[k] = (band > 0.0 && fabs(y) <= band + kBand + kEvalMargin) ? 2 : (y < 0.0 ? 1 : 0);
            unsure |= X.dec[k] == 2;
        }
        // rare: uncertain pairs, whole workgroup (skipped when there are none)
        for (int p = 0, any = __syncthreads_or(unsure ? 1 : 0); any && p < npair; ++p) {
            const int k = g + 2 * p;
            if (X.dec[k] != 2) continue;
            for (int side = 0; side < 2; ++side) {
                const int wv = X.perm[k + side];
                if (X.Eerr[wv] > 0.0) {
                    const double e = exact_energy(P, wv, red);
                    if (tid == 0) {
                        X.E[wv] = e;
                        X.Eerr[wv] = 0.0;
                        atomicAdd(&P.ctr[kCtrExactE], 1ull);
                    }
                    __syncthreads();
                }
            }
            if (tid == 0) {
                const int wa = X.perm[k], wb = X.perm[k + 1];
                const double y = X.lnu[k] - (X.E[wa] - X.E[wb]) * (X.beta[k] - X.beta[k + 1]);
                X.dec[k] = y < 0.0 ? 1 : 0;
            }
            __syncthreads();
        }
        for (int p = tid; p < npair; p += NT) {
            const int k = g + 2 * p;
            const int wa = X.perm[k], wb = X.perm[k + 1];
            const double y = X.lnu[k] - (X.E[wa] - X.E[wb]) * (X.beta[k] - X.beta[k + 1]);
            const int acc = X.dec[k];
            if (fabs(y) <= kBand) {
                atomicAdd(&P.ctr[kCtrBandedEx], 1ull);
                log_event(P, 1, m, g, k, acc, y);
            }
            // counts without a read on the critical path (each pair has one thread)
            atomicAdd(reinterpret_cast<unsigned long long *>(&P.xatt[k]), 1ull);
            if (acc) {
                X.perm[k] = wb;
                X.perm[k + 1] = wa;
                atomicAdd(reinterpret_cast<unsigned long long *>(&P.xacc[k]), 1ull);
            }
        }
        __syncthreads();
    }
    // FP32 / int tables keep tracking the energy of their own couplings (a
    // constant bound off the exact one): exact energies served this step only
    const bool keep = P.ebound > 0.0;
    for (int k = tid; k < R; k += NT) {
        P.perm[k] = X.perm[k];
        P.slot_of[X.perm[k]] = k;
        if (!keep) {
            P.E[k] = X.E[k];
            P.Eerr[k] = X.Eerr[k];
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Device-side grid barrier for the persistent (cooperative) launch.  The last
// workgroup to arrive runs the exchange, then releases the others.  Waiting
// is bounded: a time-out sets an error bit and every workgroup leaves.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned *bar_count(const Inst &P) { return reinterpret_cast<unsigned *>(&P.ctr[kCtrBarCount]); }
__device__ __forceinline__ unsigned *bar_gen(const Inst &P) { return reinterpret_cast<unsigned *>(&P.ctr[kCtrBarGen]); }

// Every thread's global writes are made visible device-wide (a release fence
// in each thread: on gfx9 one thread's fence writes back its XCD's L2, but
// stores of the other waves may not have reached it yet) before one thread
// signals; after a signal is observed, every thread takes the acquire (each
// wave's caches invalidated) before reading what other workgroups wrote.
__device__ __forceinline__ void release_all_agent()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
}
__device__ __forceinline__ void acquire_all_agent()
{
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ bool grid_arrive(const Inst &P, int32_t *flag)
{
    release_all_agent();  // spins and energies of this walker, for the exchange
    if (threadIdx.x == 0) {
        const unsigned g = __hip_atomic_load(bar_gen(P), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned old = __hip_atomic_fetch_add(bar_count(P), 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        flag[0] = old == static_cast<unsigned>(P.R) - 1u;
        flag[1] = static_cast<int32_t>(g);
    }
    acquire_all_agent();  // the last to arrive reads every walker's data
    return flag[0] != 0;
}

__device__ void grid_release(const Inst &P, int32_t *flag)
{
    release_all_agent();  // the exchange's permutation, slots, energies and counts
    if (threadIdx.x == 0) {
        __hip_atomic_store(bar_count(P), 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(bar_gen(P), static_cast<unsigned>(flag[1]) + 1u, __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

__device__ bool grid_wait(const Inst &P, int32_t *flag)
{
    if (threadIdx.x == 0) {
        const unsigned g = static_cast<unsigned>(flag[1]);
        int ok = 1;
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(bar_gen(P), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
            __builtin_amdgcn_s_sleep(8);
            if (__hip_atomic_load(&P.ctr[kCtrError], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull) {
                ok = 0;
                break;
            }
            if (wall_clock64() - t0 > kBarrierTicks) {
                atomicOr(&P.ctr[kCtrError], kErrBarrierTimeout);
                ok = 0;
                break;
            }
        }
        flag[2] = ok;
    }
    acquire_all_agent();  // the exchange's results, in every thread
    return flag[2] != 0;
}

// ---------------------------------------------------------------------------
// Lane broadcasts from a wave-uniform lane index (v_readlane, no LDS trip).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int rl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ double rl_d(double v, int l)
{
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u)), l));
    const uint32_t hi = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(static_cast<uint32_t>(u >> 32)), l));
    return __builtin_bit_cast(double, (static_cast<uint64_t>(hi) << 32) | lo);
}

// Draws of attempts [c0, c0 + cnt) of sweep n (counter (t, n, w, 0)), staged
// in LDS by the whole workgroup: site, state offset, ln u (FP64).
template <typename F>
__device__ __forceinline__ void gen_draws(const Inst &P, Walker<F> &W, int w, int64_t n, int c0, int cnt)
{
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const uint32_t t = static_cast<uint32_t>(c0 + e);
        const uint4 o = philox10(make_uint4(t, static_cast<uint32_t>(n), static_cast<uint32_t>(w), 0u), P.key0, P.key1);
        const uint32_t i = __umulhi(o.x, static_cast<uint32_t>(P.L));
        const uint32_t k = 1u + __umulhi(o.y, static_cast<uint32_t>(P.q - 1));
        W.draw[e] = i | (k << 16);
        W.dlnu[e] = log(open_unit(o.z, o.w));
    }
}

// FP64 energy difference of flipping site i from a to b in the current state,
// by wave 0 alone: the plain sum over the spins in LDS, which the chain keeps
// current (each committed flip writes its spin at once).
template <typename F>
__device__ __forceinline__ double chain_direct_dE(const Walker<F> &W, int L, int i, int a, int b)
{
    const int lane = threadIdx.x & (kWave - 1);
    double part = 0.0;
    for (int j = lane; j < L; j += kWave) {
        const int s = W.sp[j];
        int d = j - i;
        d += d < 0 ? L : 0;
        const double jv = W.J64[d];
        part += s == a ? jv : (s == b ? -jv : 0.0);
    }
    return rl_d(wave_sum(part), 0);
}

struct ChainRegs {
    double E, Eerr;     // walker energy and its error bound (workgroup-uniform)
    int64_t nupd, nacc; // flips since the last refresh; accepts this sweep (wave 0)
    double eL, errL;    // energy increments held by the accepting lanes (wave 0)
    uint32_t iters;     // guess-and-check iterations (workgroup-uniform; profiling)
};

// Phase counters of a walker, kept in thread 0's registers while profiling
// (see Phase in state.hpp) and added to Inst::phase when the launch ends.
struct PhaseAcc {
    uint64_t v[kPhN];
    uint64_t t;  // clock at the end of the last timed phase
    bool on;     // thread 0 of a profiled launch
};

__device__ __forceinline__ void ph_start(PhaseAcc &ph)
{
    if (ph.on) ph.t = clock64();
}
// Charges the cycles since the last mark to phase k.
__device__ __forceinline__ void ph_mark(PhaseAcc &ph, int k)
{
    if (ph.on) {
        const uint64_t t = clock64();
        ph.v[k] += t - ph.t;
        ph.t = t;
    }
}

__device__ __forceinline__ uint64_t lanes_below(int l) { return l >= kWave ? ~0ull : ((1ull << l) - 1ull); }

template <bool D, typename F>
__device__ __forceinline__ F coupling_to(const Walker<F> &W, int L, int i, int ip);

// Coupling J*(|i - ip|) of site i to site ip.  D: the row is doubled
// (J[k] = J*(k mod L) for k < L + span), so no wrap is needed.
template <bool D, typename F>
__device__ __forceinline__ F coupling_to(const Walker<F> &W, int L, int i, int ip)
{
    if constexpr (D) {
        return W.J[i + L - ip];
    } else {
        int d = i - ip;
        d += d < 0 ? L : 0;
        return W.J[d];  // J*(0) = 0 on the flipped site itself
    }
}

// Flip word: site (bits 0-15), old state (16-19), new state (20-23), and the
// chain's lane of the attempt in its window (24-29).
__device__ __forceinline__ uint32_t flip_word(int i, int a, int b, int lane)
{
    return static_cast<uint32_t>(i) | (static_cast<uint32_t>(a) << 16) | (static_cast<uint32_t>(b) << 20) |
           (static_cast<uint32_t>(lane) << 24);
}
__device__ __forceinline__ int fw_site(uint32_t w) { return static_cast<int>(w & 0xFFFFu); }
__device__ __forceinline__ int fw_old(uint32_t w) { return static_cast<int>((w >> 16) & 0xFu); }
__device__ __forceinline__ int fw_new(uint32_t w) { return static_cast<int>((w >> 20) & 0xFu); }
__device__ __forceinline__ int fw_lane(uint32_t w) { return static_cast<int>((w >> 24) & 0x3Fu); }
// Padding entry: site 0, state 0 -> 0 (every coefficient 0), lane 63 (no lane after it).
constexpr uint32_t kNoFlip = 63u << 24;

// One-hot code of a lane's attempt: bit a (current state), bit 16 + b (proposed).
__device__ __forceinline__ uint32_t state_code(int a, int b) { return (1u << a) | (1u << (b + 16)); }

// Change of dE = h[a][i] - h[b][i] under a flip ap -> bp of another site, in
// units of the coupling: [a=bp] - [a=ap] - [b=bp] + [b=ap], as two popcounts
// of the lane's one-hot code (the flip's masks are wave-uniform).
__device__ __forceinline__ int dE_coef(uint32_t code, uint32_t w)
{
    const uint32_t P = 1u << fw_old(w), Q = 1u << fw_new(w);  // ap == bp: both masks equal, c = 0
    // the word is wave-uniform: pin the masks to scalar registers (one SGPR operand per AND)
    const uint32_t X = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(Q | (P << 16))));
    const uint32_t Y = static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(P | (Q << 16))));
    return static_cast<int>(__popc(code & X)) - static_cast<int>(__popc(code & Y));
}

// dE of every lane after the flips lst[begin..end) (lane r of `lst` holds the
// r-th flip word; NEG: taken back out instead), in order, each applied only to the lanes after its own
// (gate: lane > fw_lane): dE = fma(c, J*(|i-ip|), dE) with c in {-2..2}, one
// rounding per flip.  The list is read at sequential indices, so the words of
// a batch are fetched independently; couplings are gathered kFlipBatch flips
// at a time and applied without branches (entries past `end` read as the
// padding word), so a batch's gathers stay in flight together.
template <typename F, bool D, bool NEG = false>
__device__ __forceinline__ void apply_list(const Walker<F> &W, int L, int i, int lane, uint32_t code, uint32_t lst,
                                           int begin, int end, double &dE)
{
    for (int p0 = begin; p0 < end; p0 += kFlipBatch) {
        uint32_t wb[kFlipBatch];
        F jb[kFlipBatch];
#pragma unroll
        for (int e = 0; e < kFlipBatch; ++e) {
            const uint32_t r = static_cast<uint32_t>(rl_i(static_cast<int>(lst), (p0 + e) & (kWave - 1)));
            wb[e] = p0 + e < end ? r : kNoFlip;
            jb[e] = coupling_to<D>(W, L, i, fw_site(wb[e]));
        }
#pragma unroll
        for (int e = 0; e < kFlipBatch; ++e) {
            const int c = dE_coef(lane > fw_lane(wb[e]) ? code : 0u, wb[e]);  // code 0: no change
            dE = fma(static_cast<double>(NEG ? -c : c), static_cast<double>(jb[e]), dE);
        }
    }
}

// The flips of the lanes in `set`, compacted in lane order: lane r of the
// result holds the r-th one's word (ds_permute moves every lane's word to its
// rank; lanes outside the set carry the padding word to the slots past them).
__device__ __forceinline__ uint32_t compact_flips(uint64_t set, int lane, uint32_t word)
{
    const bool in = (set >> lane) & 1ull;
    const int below = __popcll(set & lanes_below(lane));
    const int slot = in ? below : __popcll(set) + (lane - below);
    return static_cast<uint32_t>(__builtin_amdgcn_ds_permute(slot * 4, static_cast<int>(in ? word : kNoFlip)));
}

// Passes shorter than this run whole in every wave; longer ones are split.
constexpr int kSplitMin = 8;

// Waves that run the chain: every wave of the workgroup, or (GRP, the
// overlapped sweep) the first half, while the second half flushes.
template <bool GRP>
__device__ __forceinline__ int chain_nw()
{
    return static_cast<int>(blockDim.x / kWave) / (GRP ? 2 : 1);
}

// Barrier of the first nw waves of the workgroup through two LDS words
// (arrivals, generation): lane 0 of each wave reads the generation, arrives;
// the last to arrive clears the count and advances the generation, the others
// wait for it to advance.  The rest of the workgroup takes no part.  The wait
// is bounded: past kBarrierTicks of wall clock, or once any error bit is set,
// it sets the time-out bit in err and stops waiting (the host then reports
// the launch as failed).
__device__ __forceinline__ void group_barrier(uint32_t *bar, uint32_t nw, unsigned long long *err)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if ((threadIdx.x & (kWave - 1)) == 0) {
        const uint32_t g = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (__hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP) == nw - 1u) {
            __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            __hip_atomic_store(&bar[1], g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            const uint64_t t0 = wall_clock64();
            for (uint32_t k = 1; __hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) == g; ++k) {
                __builtin_amdgcn_s_sleep(1);
                if ((k & 4095u) == 0u &&
                    (wall_clock64() - t0 > kBarrierTicks ||
                     __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0ull)) {
                    atomicOr(err, kErrBarrierTimeout);
                    break;
                }
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

template <bool GRP, typename F>
__device__ __forceinline__ void chain_sync(const Walker<F> &W)
{
    if constexpr (GRP)
        group_barrier(W.gbar, static_cast<uint32_t>(chain_nw<true>()), W.err);
    else
        __syncthreads();
}

// dE += the corrections of flips lst[begin..end), each counted for the lanes
// past its own (gate: the caller's lane; kWave counts every flip), computed by
// the chain's waves.  Every wave holds the same 64 attempts; a short pass runs
// whole in each wave (no exchange), a long one is split into contiguous
// shares, one per wave, whose partial sums are exchanged through LDS (one
// barrier; the buffer alternates between passes so a wave still reading one
// pass's partials is never overwritten) and added in wave order, identically
// in every wave.  Rounding of the split form: each partial is a difference of
// two intermediate dE values (|.| <= 2 S), so the nw - 1 additions of
// partials and the final addition add at most 2 units of 2 unit, counted in ex.
template <typename F, bool D, bool NEG = false, bool GRP = false>
__device__ __forceinline__ void add_flips_wg(const Walker<F> &W, int L, int i, int gate, uint32_t code, uint32_t lst,
                                             int begin, int end, double &dE, int &ex, int &pbuf)
{
    const int nw = chain_nw<GRP>(), wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int n = end - begin;
    if (nw == 1 || n < kSplitMin) {
        apply_list<F, D, NEG>(W, L, i, gate, code, lst, begin, end, dE);
        return;
    }
    const int per = (n + nw - 1) / nw;
    const int b0 = min(end, begin + wv * per), b1 = min(end, b0 + per);
    double part = 0.0;
    apply_list<F, D, NEG>(W, L, i, gate, code, lst, b0, b1, part);
    double *xp = W.xpart + pbuf * nw * kWave;
    xp[wv * kWave + lane] = part;
    chain_sync<GRP>(W);
    double tot = xp[lane];
    for (int k = 1; k < nw; ++k) tot += xp[k * kWave + lane];
    pbuf ^= 1;
    dE += tot;
    ex += 2;
}

// Field of state c at site i from the table (table units, in FP64): rows
// 0 .. q-2 are stored, row q-1 is the coupling sum of the table's couplings
// minus the others (the q fields of a site sum to it).
template <typename F>
__device__ __forceinline__ double tab_entry(const Inst &P, const Walker<F> &W, int c, int i)
{
    const int L = P.L, r = P.q - 1;
    if (c < r) return static_cast<double>(W.h[c * L + i]);
    double v = P.hsum;
    for (int k = 0; k < r; ++k) v -= static_cast<double>(W.h[k * L + i]);
    return v;
}

// h[a][i] - h[b][i] from the table.  Up to eight stored rows (q <= 9) every
// lane reads them all at once (independent loads, in flight together: the
// table may be in HBM) and picks its two entries, with no divergent branch in
// the chain's serial path.
template <typename F>
__device__ __forceinline__ double tab_dE(const Inst &P, const Walker<F> &W, int a, int b, int i)
{
    const int L = P.L, r = P.q - 1;
    if (r <= 3) {  // the short form: three loads, four selects
        const double v0 = static_cast<double>(W.h[i]);
        const double v1 = r > 1 ? static_cast<double>(W.h[L + i]) : 0.0;
        const double v2 = r > 2 ? static_cast<double>(W.h[2 * L + i]) : 0.0;
        const double last = ((P.hsum - v0) - v1) - v2;  // subtracting the zeros is exact
        const double ha = a == r ? last : (a == 0 ? v0 : (a == 1 ? v1 : v2));
        const double hb = b == r ? last : (b == 0 ? v0 : (b == 1 ? v1 : v2));
        return ha - hb;
    }
    if (r <= 8) {
        double v[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = k < r ? static_cast<double>(W.h[k * L + i]) : 0.0;
        double last = P.hsum;
#pragma unroll
        for (int k = 0; k < 8; ++k) last -= v[k];  // subtracting the zeros is exact
        double ha = last, hb = last;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            ha = a == k && k < r ? v[k] : ha;
            hb = b == k && k < r ? v[k] : hb;
        }
        return ha - hb;
    }
    return tab_entry(P, W, a, i) - tab_entry(P, W, b, i);
}

// dE = h[a][i] - h[b][i] as the chain sees it: the two table entries (window
// start) plus the window's flips 0..np-1 (all earlier than any live lane).
template <typename F, bool D>
__device__ __forceinline__ double dE_now(const Inst &P, const Walker<F> &W, int L, int a, int b, int i, int np, int &ex,
                                         int &pbuf)
{
    const int lane = threadIdx.x & (kWave - 1);
    double dE = tab_dE(P, W, a, b, i);
    const uint32_t pv = lane < np ? W.pend[lane] : kNoFlip;
    ex = 0;
    add_flips_wg<F, D>(W, L, i, kWave, state_code(a, b), pv, 0, np, dE, ex, pbuf);
    return dE;
}

// Overlapped sweep: a window's fields for every state at its sites, read
// before the previous window's flush starts, and that window's flip list.
struct Snap {
    double v[4];     // h[c][i], c < q <= 4 (table units)
    uint32_t prev;   // lane r: the previous window's r-th flip word
    int nprev;
};

__device__ __forceinline__ double sel4(const double (&v)[4], int k)
{
    return k == 0 ? v[0] : (k == 1 ? v[1] : (k == 2 ? v[2] : v[3]));
}

// Direct energy changes (no field table): dE of every lane's attempt,
// sum_j J*(|i-j|) ([s_j = a] - [s_j = b]), over the spins in LDS (current: the
// chain writes each committed flip's spin at once), in FP64.  The 64 sums
// are split between the waves, each wave taking a contiguous share of the
// attempts with all its lanes running over the sites, and exchanged through
// LDS (one barrier); every wave ends with the same 64 values.
template <typename F>
__device__ __forceinline__ double direct_dE_window(const Walker<F> &W, int L, int i, int a, int b, int &pbuf)
{
    const int nw = blockDim.x / kWave, wv = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
    const int per = (kWave + nw - 1) / nw;
    const int g0 = wv * per, g1 = min(kWave, g0 + per);
    double mine = 0.0;
    // two attempts per pass over the spins (each spin read once for both)
    for (int g = g0; g < g1; g += 2) {
        const int h = min(g + 1, g1 - 1);  // an odd share repeats its last attempt
        const int i0 = rl_i(i, g), a0 = rl_i(a, g), b0 = rl_i(b, g);
        const int i1 = rl_i(i, h), a1 = rl_i(a, h), b1 = rl_i(b, h);
        double p0 = 0.0, p1 = 0.0;
        for (int j = lane; j < L; j += kWave) {
            const int s = W.sp[j];
            int d0 = j - i0, d1 = j - i1;
            d0 += d0 < 0 ? L : 0;
            d1 += d1 < 0 ? L : 0;
            const double v0 = W.J64[d0], v1 = W.J64[d1];
            p0 += s == a0 ? v0 : (s == b0 ? -v0 : 0.0);
            p1 += s == a1 ? v1 : (s == b1 ? -v1 : 0.0);
        }
        const double t0 = wave_sum(p0), t1 = wave_sum(p1);
        mine = lane == g ? t0 : mine;
        mine = lane == h ? t1 : mine;
    }
    if (nw == 1) return mine;
    double *xp = W.xpart + pbuf * nw * kWave;
    if (lane >= g0 && lane < g1) xp[lane] = mine;
    __syncthreads();
    const double r = xp[lane];
    pbuf ^= 1;
    return r;
}

// The chain through attempts [t0, t0 + 64) (lanes past `cend` idle), run by
// every wave of the workgroup on the same 64 attempts: all decisions are taken
// identically in each wave, the long correction passes are split between the
// waves (add_flips_wg), and the shared results (flip list, spins) are written
// by every wave with the same values; counters, events and energy increments
// are kept by wave 0 alone.  Each lane keeps its attempt's energy change
// dE = h[a][i] - h[b][i] (a the current state of its site, b the proposed
// one), read from the table once.
// The sequential chain is resolved by guess and check: every attempt that is
// a sure accept under the current dE is guessed to be accepted; the guess
// stops at the first later attempt on a site a guessed flip changed, whose
// state the guess cannot know; the guessed flips before it are applied, in
// order, to the later lanes' dE.  Each lane then re-decides with exactly the
// guessed flips before it and its own bound.  Up to the first lane whose
// decision differs from the guess, every lane saw precisely the flips the
// sequential chain would have accepted before it, so that prefix is
// committed; the differing lane is decided (near-threshold ones by the FP64
// direct sum) and the later lanes' dE are rebuilt from the committed flips.
// Committed flips write their spins at once; a later lane whose site changed
// takes the new state and re-derives dE from the table and the window's
// flips.  Energy increments stay in the accepting lane (eL, errL) and are
// summed at the end of the sweep.
//
// Rounding: dE starts as the difference of two table entries (each within
// init + nupd * unit of exact) and takes at most 2 unit of rounding per applied
// flip, so Bd = 2 (init + nupd * unit) grown by 2 unit per flip bounds its
// error exactly as for two separately kept fields; a split pass adds `ex`
// more such units per lane.
template <typename F, bool D, bool DIR, bool GRP = false>
__device__ __forceinline__ void chain_window(const Inst &P, Walker<F> &W, int w, int64_t n, double beta_r, int t0,
                                             int c0, int cend, ChainRegs &cr, int &pbuf, const Snap *snap = nullptr,
                                             PhaseAcc *php = nullptr)
{
    // profiled runs: thread 0 charges each step of an iteration to its counter
    const bool pon = php && php->on;
    uint64_t tq = pon ? clock64() : 0;
    auto mark = [&](int k) {
        if (pon) {
            const uint64_t t = clock64();
            php->v[k] += t - tq;
            tq = t;
        }
    };
    constexpr bool kF64 = sizeof(F) == sizeof(double);
    constexpr bool kI32 = table_prec<F>() == kPrecI32;
    const int L = P.L, q = P.q, lane = threadIdx.x & (kWave - 1);
    const bool lead = threadIdx.x < kWave;  // wave 0 keeps counters, events and energy increments
    uint32_t *sfirst = W.sfirst ? W.sfirst + (threadIdx.x / kWave) * L : nullptr;
    const uint64_t mine_below = lanes_below(lane);
    const int ta = t0 + lane;
    const bool valid = ta < cend;
    const uint32_t dr = valid ? W.draw[ta - c0] : 0u;
    const int i = static_cast<int>(dr & 0xFFFFu);
    const int kk = static_cast<int>(dr >> 16);
    const double lnu = valid ? W.dlnu[ta - c0] : 0.0;
    int a = W.sp[i];
    int b = a + kk;
    b -= b >= q ? q : 0;
    double dE;
    int ex = 0;  // extra roundings in this lane's dE, in units of 2 unit
    if constexpr (DIR) {
        dE = direct_dE_window(W, L, i, a, b, pbuf);
    } else if constexpr (GRP) {
        // the snapshot (the table before the previous window's flush) plus that
        // window's flips, all earlier than this window's attempts
        dE = sel4(snap->v, a) - sel4(snap->v, b);
        add_flips_wg<F, D, false, GRP>(W, L, i, kWave, state_code(a, b), snap->prev, 0, snap->nprev, dE, ex, pbuf);
    } else {
        dE = tab_dE(P, W, a, b, i);
    }
    uint32_t code = state_code(a, b);
    uint64_t live = ballot(valid);
    int np = 0;
    double Bd = P.bound_rows * (P.bound_init + static_cast<double>(cr.nupd) * P.bound_unit) + P.bound_impl;
    const double dBd = 2.0 * P.bound_unit;
    const double tfix = kBand + kEvalMargin;
    // dE, its bounds and eL are in table units (real value = qscale * units; the
    // scale is a power of two, 1 for FP tables), so beta is taken per unit
    const double beta = beta_r * P.qscale;
    while (live) {
        ++cr.iters;
        const uint32_t pk = flip_word(i, a, b, lane);
        // guess: the sure accepts under the current dE
        uint64_t S = ballot(beta * dE + lnu < -(beta * Bd + tfix)) & live;
        const bool inS0 = (S >> lane) & 1ull;
        // the first lane after a guessed flip on its own site.  A guessed flip
        // at or past that lane only meets lanes past it, so testing against
        // all of S finds the same first lane as stopping there would.
        uint64_t dm = 0;
        if (S) {
            if (sfirst) {  // this wave's per-site table: the first guessed lane on each site
                if (inS0) atomicMin(&sfirst[i], static_cast<uint32_t>(lane));
                const uint32_t f0 = sfirst[i];
                dm = ballot(valid && f0 < static_cast<uint32_t>(lane));
                if (inS0) sfirst[i] = kWave;
            } else {
                for (uint64_t sm = S; sm; sm &= sm - 1ull) {
                    const int p = static_cast<int>(__builtin_ctzll(sm));
                    dm |= ballot(valid && lane > p && i == rl_i(i, p));
                }
            }
        }
        const int hz = dm ? static_cast<int>(__builtin_ctzll(dm)) : kWave;
        S &= lanes_below(hz);
        const double dE0 = dE;
        const int ex0 = ex;
        const uint32_t lst = compact_flips(S, lane, pk);  // lane r: the r-th guessed flip
        mark(kPhCGuess);
        add_flips_wg<F, D, false, GRP>(W, L, i, lane, code, lst, 0, __popcll(S), dE, ex, pbuf);
        mark(kPhCCorr);
        // check: each lane decides with the guessed flips before it
        const double x = beta * dE + lnu;
        const int r = __popcll(S & mine_below);
        const double Bdl = Bd + static_cast<double>(r + ex) * dBd;
        const double trig = beta * Bdl + tfix;
        const bool inS = (S >> lane) & 1ull;
        const bool sure = x < -trig, rej = x > trig;
        const uint64_t V = ballot(inS ? !sure : !rej) & live & lanes_below(hz);
        const int m = V ? static_cast<int>(__builtin_ctzll(V)) : hz;
        const uint64_t C = S & lanes_below(m);
        if ((C >> lane) & 1ull) {  // committed lanes have distinct sites
            W.pend[np + r] = pk;
            W.sp[i] = static_cast<uint8_t>(b);
        }
        if (lead && ((C >> lane) & 1ull)) {
            atomicAdd(&W.cnt[a], -1);
            atomicAdd(&W.cnt[b], 1);
            // FP32 tables take E from the flush's sums; int tables' dE is exact
            // in their quantised couplings (a constant bound covers the rest)
            if (kF64 || DIR || kI32) cr.eL += dE;
            if (kF64 || DIR) cr.errL += Bdl;
        }
        const int nc = __popcll(C);
        np += nc;
        if (!DIR) cr.nupd += nc;  // flips the table will take (none without a table)
        cr.nacc += nc;
        Bd += static_cast<double>(nc) * dBd;
        mark(kPhCCheck);
        if (V) {
            // lane m holds exactly the committed flips: decide it
            const uint32_t pk_m = static_cast<uint32_t>(rl_i(static_cast<int>(pk), m));
            const int i_m = fw_site(pk_m), a_m = fw_old(pk_m), b_m = fw_new(pk_m);
            bool accept = (ballot(sure) >> m) & 1ull;
            double dEm = rl_d(dE, m), errm = Bd + static_cast<double>(rl_i(ex, m)) * dBd;
            if (!accept && !((ballot(rej) >> m) & 1ull)) {
                // |x| inside the trigger band: decide with the FP64 direct sum
                const double d64 = chain_direct_dE(W, L, i_m, a_m, b_m);
                const double x64 = beta_r * d64 + rl_d(lnu, m);
                accept = x64 < 0.0;
                if constexpr (!kI32) {  // int tables keep the energy of their own couplings
                    dEm = d64;
                    errm = 0.0;
                }
                if (lead && lane == 0) {
                    atomicAdd(&P.ctr[kCtrRecheck], 1ull);
                    if (fabs(x64) <= kBand) {
                        atomicAdd(&P.ctr[kCtrBandedMet], 1ull);
                        log_event(P, 0, w, n, t0 + m, accept ? 1 : 0, x64);
                    }
                }
            }
            // rebuild the later lanes' dE from the committed flips (the list's
            // first nc): re-add them to dE0, or, when fewer guessed flips lie
            // past m, take those back out of the guess.  A lane past m then
            // keeps the roundings of its r - nc removed flips twice (added
            // and taken out), 2 (r - nc) more units beyond the committed ones.
            const int ns = __popcll(S);
            if (nc <= ns - nc) {
                dE = dE0;
                ex = ex0;
                add_flips_wg<F, D, false, GRP>(W, L, i, lane, code, lst, 0, nc, dE, ex, pbuf);
            } else {
                add_flips_wg<F, D, true, GRP>(W, L, i, lane, code, lst, nc, ns, dE, ex, pbuf);
                ex += 2 * max(0, r - nc);
            }
            if (accept) {
                if (lane == m) {
                    W.pend[np] = pk_m;
                    W.sp[i_m] = static_cast<uint8_t>(b_m);
                }
                if (lead && lane == m) {
                    atomicAdd(&W.cnt[a_m], -1);
                    atomicAdd(&W.cnt[b_m], 1);
                    if (kF64 || DIR || kI32) cr.eL += dEm;
                    if (kF64 || DIR) cr.errL += errm;
                }
                ++np;
                if (!DIR) ++cr.nupd;
                ++cr.nacc;
                Bd += dBd;
                const int c = dE_coef(lane > m ? code : 0u, pk_m);
                dE = fma(static_cast<double>(c), static_cast<double>(coupling_to<D>(W, L, i, i_m)), dE);
            }
            live &= ~lanes_below(m + 1);
        } else {
            live &= ~lanes_below(hz);
        }
        mark(kPhCResolve);
        // a later lane whose site's spin changed: new current state, dE re-derived
        const int sn = W.sp[i];
        const bool redo = ((live >> lane) & 1ull) && sn != a;
        if (ballot(redo)) {
            int b2 = sn + kk;
            b2 -= b2 >= q ? q : 0;
            int ex2 = 0;
            double dE2;
            if constexpr (DIR) {
                // direct sums for the lanes that need them, one by one, in every wave alike
                dE2 = 0.0;
                for (uint64_t rm = ballot(redo); rm; rm &= rm - 1ull) {
                    const int g = static_cast<int>(__builtin_ctzll(rm));
                    const double t = chain_direct_dE(W, L, rl_i(i, g), rl_i(sn, g), rl_i(b2, g));
                    dE2 = lane == g ? t : dE2;
                }
            } else if constexpr (GRP) {
                // snapshot + the previous window's flips + this window's first np
                const int a2 = redo ? sn : a, bb = redo ? b2 : b;
                dE2 = sel4(snap->v, a2) - sel4(snap->v, bb);
                add_flips_wg<F, D, false, GRP>(W, L, i, kWave, state_code(a2, bb), snap->prev, 0, snap->nprev, dE2, ex2,
                                               pbuf);
                const uint32_t pv = lane < np ? W.pend[lane] : kNoFlip;
                add_flips_wg<F, D, false, GRP>(W, L, i, kWave, state_code(a2, bb), pv, 0, np, dE2, ex2, pbuf);
            } else {
                dE2 = dE_now<F, D>(P, W, L, redo ? sn : a, redo ? b2 : b, i, np, ex2, pbuf);
            }
            if (redo) {
                a = sn;
                b = b2;
                code = state_code(a, b);
                dE = dE2;
                ex = ex2;
            }
        }
        mark(kPhCRedo);
        // every wave has finished reading this iteration's spins before any
        // wave writes the next iteration's commits
        if (chain_nw<GRP>() > 1) chain_sync<GRP>(W);
        mark(kPhCSync);
    }
    if (lead && lane == 0) W.cs->np[(t0 / kWave) & 1] = np;
}

// Threads tid of NT (the whole workgroup, or the flush waves of an overlapped
// sweep): apply the window's np flips to the table.  Each thread
// owns M sites per pass and applies the flips to them in order, so no
// barrier is needed between flips.  QT > 0 (q <= QT, QT = 4, 6 or 8): the
// sites' fields of the rows the window's flips touch sit in registers for the
// pass (one table read and write per field; untouched rows are neither read
// nor written, which matters when the table is in HBM) and every flip is
// applied to all QT rows as fma(coef, J, h) with a wave-uniform coefficient (-1, 0 or +1:
// from a table by flip kind for QT = 4, computed from the flip's states
// otherwise), which rounds exactly as h - J or h + J and leaves an untouched
// row's zeros alone; QT = 0 (larger q): per batch of flips, the rows the batch
// touches are updated one after another, each entry read and written once per
// batch, the next row's read in flight during this row's update.  Int tables
// are updated in FP64 registers, exact for their integer values (|h| < 2^31):
// the same fma form, no branch per flip.  The couplings of kFlipBatch flips are
// gathered before they are applied; with a doubled coupling row (D) one address
// serves a flip's kFlushM gathers.  With an FP32 table the same pass forms
// every flip's energy change in FP64 from the FP32 couplings it already holds,
// sum_j J32(|j-i|)[delta(a, s_j) - delta(b, s_j)], over the spins as they were
// just before it (partial sums per thread; the window-start spins are
// recovered from the flip list, since the chain has already written the new
// ones); its error against the exact change is at most the bound_flipE the
// caller charges per flip.
template <typename F, int QT, bool D>
__device__ __forceinline__ void flush_window(const Inst &P, Walker<F> &W, int np, double &part, int tid, int NT,
                                             int nrows)
{
    constexpr int QR = QT > 0 ? QT : 1;  // rows held in registers (q <= QT)
    constexpr int M = kFlushM;             // register slots per thread
    constexpr int B = kFlipBatch;
    constexpr bool kF32 = table_prec<F>() == kPrecF32;
    constexpr bool kI32 = table_prec<F>() == kPrecI32;
    using RT = typename std::conditional<kI32, double, F>::type;  // register arithmetic
    const int L = P.L, lane = tid & (kWave - 1);  // threads tid of NT (whole waves) take part
    static_assert(kMaxSweepThreads <= 256 && kMaxJobThreads <= 256, "M sites per thread assume <= 256 threads");
    const uint32_t pv = lane < np ? W.pend[lane] : kNoFlip;  // the chain already wrote the spins
    // rows the window's flips touch (wave-uniform bits)
    uint32_t touched = 0;
    if constexpr (QT > 0) {
        const uint32_t mine = lane < np ? ((1u << fw_old(pv)) | (1u << fw_new(pv))) : 0u;
#pragma unroll
        for (int c = 0; c < QT; ++c) touched |= ballot((mine >> c) & 1u) ? (1u << c) : 0u;
        touched &= (1u << nrows) - 1u;  // rows the table stores
    }
    for (int jb = (tid / kWave) * kWave * M; jb < L; jb += NT * M) {
        const int j0 = jb + lane;
        int jm[M];
        bool ok[M];
        RT hr[QR][M];
        int sr[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int j = j0 + m * kWave;
            ok[m] = j < L;
            jm[m] = ok[m] ? j : 0;
            sr[m] = (kF32 && ok[m]) ? W.sp[j] : -1;
        }
        if (kF32) {  // back to the window's start: the first flip of a site holds its old state
            for (int p = np - 1; p >= 0; --p) {
                const uint32_t pk = static_cast<uint32_t>(rl_i(static_cast<int>(pv), p));
                const int ip = fw_site(pk), ap = fw_old(pk);
#pragma unroll
                for (int m = 0; m < M; ++m) sr[m] = (ok[m] && jm[m] == ip) ? ap : sr[m];
            }
        }
#pragma unroll
        for (int c = 0; c < QT; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m)
                hr[c][m] = (((touched >> c) & 1u) && ok[m]) ? static_cast<RT>(W.h[c * L + jm[m]]) : RT(0);
        (void)hr;
        const F *Jrow = W.J + (j0 + L);  // D: coupling of site j0 + 64 m to site ip is Jrow[64 m - ip]
        // the batches of the window's flips; kTab: coefficient rows from the
        // LDS table (the two- and four-row forms run only for q <= 4, every
        // state below 4), else computed from the flip's states
        auto batches = [&](auto tab) {
            constexpr bool kTab = decltype(tab)::value;
            for (int p0 = 0; p0 < np; p0 += B) {
                uint32_t pkb[B];
                RT g[B][M];
#pragma unroll
                for (int e = 0; e < B; ++e) {
                    // p0 + e <= 63; lanes past np hold the no-flip word
                    pkb[e] = static_cast<uint32_t>(rl_i(static_cast<int>(pv), p0 + e));
                    const int ip = fw_site(pkb[e]);
#pragma unroll
                    for (int m = 0; m < M; ++m) {
                        if constexpr (D) {
                            g[e][m] = static_cast<RT>(Jrow[m * kWave - ip]);
                        } else {
                            int d = jm[m] - ip;
                            d += d < 0 ? L : 0;
                            g[e][m] = static_cast<RT>(W.J[d]);
                        }
                    }
                }
                // no branch per flip: padding entries have all coefficients 0
                if constexpr (kTab) {
#pragma unroll
                    for (int e = 0; e < B; ++e) {
                        const F *kc = W.ctab + ((pkb[e] >> 16) & 0x3Fu) * 4;  // one broadcast row per flip
#pragma unroll
                        for (int c = 0; c < QT; ++c) {
                            const F k = kc[c];
#pragma unroll
                            for (int m = 0; m < M; ++m)
                                hr[c][m] = fma(k, g[e][m], hr[c][m]);
                        }
                    }
                } else if constexpr (QT > 0) {
                    // every row, flip by flip (no branch: QT * M independent fma per flip)
#pragma unroll
                    for (int e = 0; e < B; ++e) {
                        const int ap = fw_old(pkb[e]), bp = fw_new(pkb[e]);
#pragma unroll
                        for (int c = 0; c < QT; ++c) {
                            const RT k = flip_coef<RT>(c, ap, bp);  // wave-uniform; padding: 0
#pragma unroll
                            for (int m = 0; m < M; ++m) hr[c][m] = fma(k, g[e][m], hr[c][m]);
                        }
                    }
                }
                if (kF32) {
#pragma unroll
                    for (int e = 0; e < B; ++e) {
                        const bool real = p0 + e < np;
                        const int ip = fw_site(pkb[e]), ap = fw_old(pkb[e]), bp = fw_new(pkb[e]);
#pragma unroll
                        for (int m = 0; m < M; ++m) {
                            const int sj = sr[m];
                            const double gv = static_cast<double>(g[e][m]);
                            part += (real && sj == ap) ? gv : ((real && sj == bp) ? -gv : 0.0);
                            sr[m] = (real && ok[m] && jm[m] == ip) ? bp : sj;
                        }
                    }
                }
                if constexpr (QT == 0) {
                    // larger q: the rows this batch touches, one after another; each
                    // entry is read once, takes the batch's flips in order and is
                    // written once, and the next row's read is issued before this
                    // row's write (no write-to-read wait; the table may be in HBM)
                    uint32_t rows = 0;
#pragma unroll
                    for (int e = 0; e < B; ++e) rows |= (1u << fw_old(pkb[e])) | (1u << fw_new(pkb[e]));
                    // stored rows only; rows != 0: a flip touches two states, at
                    // most one of them the implicit last, and padding touches row 0
                    rows &= (1u << nrows) - 1u;
                    int c = static_cast<int>(__builtin_ctz(rows));
                    RT vn[M];
#pragma unroll
                    for (int m = 0; m < M; ++m) vn[m] = ok[m] ? static_cast<RT>(W.h[c * L + jm[m]]) : RT(0);
                    while (c >= 0) {
                        RT v[M];
#pragma unroll
                        for (int m = 0; m < M; ++m) v[m] = vn[m];
                        rows &= rows - 1u;
                        const int cn = rows ? static_cast<int>(__builtin_ctz(rows)) : -1;
                        if (cn >= 0) {
#pragma unroll
                            for (int m = 0; m < M; ++m) vn[m] = ok[m] ? static_cast<RT>(W.h[cn * L + jm[m]]) : RT(0);
                        }
#pragma unroll
                        for (int e = 0; e < B; ++e) {
                            const RT k = flip_coef<RT>(c, fw_old(pkb[e]), fw_new(pkb[e]));  // padding: 0
#pragma unroll
                            for (int m = 0; m < M; ++m) v[m] = fma(k, g[e][m], v[m]);
                        }
#pragma unroll
                        for (int m = 0; m < M; ++m)
                            if (ok[m]) W.h[c * L + jm[m]] = static_cast<F>(v[m]);
                        c = cn;
                    }
                }
            }
        };
        batches(std::integral_constant<bool, (QT == 4 || QT == 2) && !kI32>{});
#pragma unroll
        for (int c = 0; c < QT; ++c)
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (((touched >> c) & 1u) && ok[m]) W.h[c * L + jm[m]] = static_cast<F>(hr[c][m]);
    }
}

// One sweep of walker w at sweep index n.  Returns this thread's part of the
// energy change (FP32 table: the flush's sums; zero otherwise).  PL: the table
// in LDS (with a doubled coupling row) or in HBM, whose windows' flips the
// flush applies, or no table, the chain taking its energy changes from direct
// sums over the spins.
template <typename F, int QT, int PL>
__device__ __forceinline__ double sweep_walker(const Inst &P, Walker<F> &W, int w, int64_t n, double beta, ChainRegs &cr,
                                               PhaseAcc &ph)
{
    constexpr bool D = PL == kPlLds, TAB = PL != kPlDirect;
    const int L = P.L;
    double part = 0.0;
    int pbuf = 0;
    for (int c0 = 0; c0 < L; c0 += W.chunk) {
        const int cend = min(L, c0 + W.chunk);
        ph_start(ph);
        gen_draws<F>(P, W, w, n, c0, cend - c0);
        __syncthreads();
        ph_mark(ph, kPhDraw);
        for (int t0 = c0; t0 < cend; t0 += kWave) {
            chain_window<F, D, !TAB>(P, W, w, n, beta, t0, c0, cend, cr, pbuf, nullptr, &ph);
            __syncthreads();
            ph_mark(ph, kPhChain);
            const int np = W.cs->np[(t0 / kWave) & 1];
            if (TAB && np > 0) {  // without a table the chain works from direct sums: nothing to flush
                flush_window<F, QT, D>(P, W, np, part, threadIdx.x, blockDim.x, P.q - 1);
                __syncthreads();
                ph_mark(ph, kPhFlush);
                if (ph.on) ++ph.v[kPhFlushes];
            }
            if (ph.on) {
                ++ph.v[kPhWindows];
                ph.v[kPhFlips] += static_cast<uint64_t>(np);
            }
        }
    }
    return part;
}

// One sweep with the chain and the flush overlapped (table in LDS, q <= 4,
// the whole sweep's draws in one chunk; FP64 and int32 tables, whose flush
// reads no spins).  The first half of the waves runs the chain, the second
// half flushes.  Step s: the chain waves read window s's fields for every state
// at its sites (the table as of window s - 2's flush); one workgroup barrier;
// then the flush waves apply window s - 1's flips while the chain waves add
// those same flips to their energy changes and run window s; one more barrier.
// A window costs about the larger of its chain and the previous window's
// flush instead of their sum.
template <typename F, int QT>
__device__ __forceinline__ double sweep_walker_ov(const Inst &P, Walker<F> &W, int w, int64_t n, double beta,
                                                  ChainRegs &cr, PhaseAcc &ph)
{
    const int L = P.L, q = P.q, lane = threadIdx.x & (kWave - 1);
    const int nc = chain_nw<true>();
    const bool chainw = static_cast<int>(threadIdx.x / kWave) < nc;
    uint32_t *const pend0 = W.pend;  // [2][64]: the flip lists of even and odd windows
    double part = 0.0;
    int pbuf = 0;
    ph_start(ph);
    gen_draws<F>(P, W, w, n, 0, L);
    __syncthreads();
    ph_mark(ph, kPhDraw);
    const int nwin = (L + kWave - 1) / kWave;
    int np_prev = 0;
    // the chain's waves issue first on their SIMDs: it is the serial path
    if (chainw) __builtin_amdgcn_s_setprio(3);
    for (int s = 0; s <= nwin; ++s) {
        const int t0 = s * kWave;
        Snap sn;
        sn.nprev = np_prev;
        sn.prev = lane < np_prev ? pend0[((s - 1) & 1) * kWave + lane] : kNoFlip;
        if (chainw && s < nwin) {
            const int ta = t0 + lane;
            const int i = ta < L ? static_cast<int>(W.draw[ta] & 0xFFFFu) : 0;
            double last = P.hsum;  // row q-1: the coupling sum minus the stored rows
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                sn.v[c] = c < q - 1 ? static_cast<double>(W.h[c * L + i]) : 0.0;
                last -= sn.v[c];
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) sn.v[c] = c == q - 1 ? last : sn.v[c];
        }
        __syncthreads();  // the snapshot is read before the flush below writes the table
        if (chainw) {
            if (s < nwin) {
                W.pend = pend0 + (s & 1) * kWave;
                chain_window<F, true, false, true>(P, W, w, n, beta, t0, 0, L, cr, pbuf, &sn);
            }
        } else if (np_prev > 0) {
            if (ph.on) ph.t = clock64();
            Walker<F> Wf = W;
            Wf.pend = pend0 + ((s - 1) & 1) * kWave;
            flush_window<F, QT, true>(P, Wf, np_prev, part, threadIdx.x - nc * kWave, nc * kWave, P.q - 1);
            ph_mark(ph, kPhFlush);
            if (ph.on) ++ph.v[kPhFlushes];
        }
        __syncthreads();  // window s decided, window s - 1 flushed
        np_prev = s < nwin ? W.cs->np[s & 1] : 0;
        if (ph.on && threadIdx.x == 0) {
            ph_mark(ph, kPhChain);
            if (s < nwin) {
                ++ph.v[kPhWindows];
                ph.v[kPhFlips] += static_cast<uint64_t>(np_prev);
            }
        }
    }
    if (chainw) __builtin_amdgcn_s_setprio(0);
    W.pend = pend0;
    return part;
}

template <typename F>
__device__ __forceinline__ void record_sweep(const Inst &P, const Walker<F> &W, int w, int slot, int64_t n, double E, int64_t nacc)
{
    if (threadIdx.x != 0) return;
    int nmax = 0;
    for (int k = 0; k < P.q; ++k) nmax = max(nmax, W.cnt[k]);
    const double M = (static_cast<double>(P.q) * nmax / P.L - 1.0) / (P.q - 1);
    const int R = P.R;
    const double e2 = E * E, m2 = M * M;
    P.acc6[0 * R + slot] += E;
    P.acc6[1 * R + slot] += e2;
    P.acc6[2 * R + slot] += e2 * e2;
    P.acc6[3 * R + slot] += M;
    P.acc6[4 * R + slot] += m2;
    P.acc6[5 * R + slot] += m2 * m2;
    P.fatt[slot] += P.L;
    P.facc[slot] += nacc;
    P.Mw[w] = M;
    if (n < P.ser_cap) {
        P.serE[n * R + slot] = E;
        P.serM[n * R + slot] = M;
    }
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
// Sum of the couplings S = sum_{r=1}^{L-1} J*(r) in FP64, by one whole wave in
// a fixed order (lane-strided partial sums, then the butterfly reduction, which
// leaves the same value in every lane), so that every caller gets the same
// bits whatever its workgroup size.
template <typename T>
__device__ __forceinline__ double coupling_sum_wave(const T *J, int L)
{
    const int lane = threadIdx.x & (kWave - 1);
    double part = 0.0;
    for (int r = 1 + lane; r < L; r += kWave) part += static_cast<double>(J[r]);
    return wave_sum(part);
}

// sum_r |J*(r) - scale Jr(r)|, a coupling table's total rounding, by one wave.
template <typename T>
__device__ __forceinline__ double coupling_error_wave(const double *J64, const T *Jr, double scale, int L)
{
    const int lane = threadIdx.x & (kWave - 1);
    double part = 0.0;
    for (int r = 1 + lane; r < L; r += kWave) part += fabs(J64[r] - scale * static_cast<double>(Jr[r]));
    return wave_sum(part) * 1.001;
}

// After the couplings J64/J32 are written (the whole workgroup, at least one
// wave): the quantised couplings Jq(r) = rint(J*(r) 2^k), k the largest with
// S 2^k + L < 2^31 - 2 (no field of an int table can then overflow), and the
// table bounds at P.bnd for precision prec (lane 0 of wave 0 writes them),
// with the coupling sum of the table's own couplings (its implicit row).
__device__ void setup_couplings(const Inst &P, int prec)
{
    __shared__ double s_scale;
    const int L = P.L;
    double S = 0.0;
    if (threadIdx.x < kWave) {
        S = coupling_sum_wave(P.J64, L);
        if (threadIdx.x == 0) {
            int k = 0;
            while (k < 60 && S * ldexp(1.0, k + 1) + static_cast<double>(L) < 2147483646.0) ++k;
            s_scale = ldexp(1.0, k);
        }
    }
    __syncthreads();
    const double up = s_scale;
    int32_t *Jq = const_cast<int32_t *>(P.Jq);
    for (int r = threadIdx.x; r < L; r += blockDim.x) Jq[r] = static_cast<int32_t>(rint(P.J64[r] * up));
    __syncthreads();
    if (threadIdx.x < kWave) {
        const double D32 = coupling_error_wave(P.J64, P.J32, 1.0, L);
        const double Dq = coupling_error_wave(P.J64, P.Jq, 1.0 / up, L);
        // int sums are exact (|sum| < 2^31); FP32 couplings are summed in FP64
        const double Stab = prec == kPrecI32 ? coupling_sum_wave(P.Jq, L)
                                             : (prec == kPrecF32 ? coupling_sum_wave(P.J32, L) : S);
        if (threadIdx.x == 0) *P.bnd = table_bounds(S, P.J64[1], D32, Dq, L, prec, 1.0 / up, P.q, Stab);
    }
    __syncthreads();
}

// Ladder, quantised couplings and table bounds of a fresh instance (after
// k_jstar): beta_k = 1/T_k from the temperatures at T (device memory), the
// identity slot permutation, and setup_couplings.  One workgroup.
static __global__ void k_setup(Inst P, const double *__restrict__ T, int32_t prec)
{
    for (int k = threadIdx.x; k < P.R; k += blockDim.x) {
        const_cast<double *>(P.beta)[k] = 1.0 / T[k];
        P.perm[k] = k;
        P.slot_of[k] = k;
    }
    setup_couplings(P, prec);
}

// Current energy and magnetisation by temperature slot (E_slot[k] =
// E[perm[k]]), for a caller that copies observables without host staging.
static __global__ void k_obs_by_slot(Inst P, double *__restrict__ Eslot, double *__restrict__ Mslot)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P.R; k += gridDim.x * blockDim.x) {
        const int w = P.perm[k];
        Eslot[k] = P.E[w];
        Mslot[k] = P.Mw[w];
    }
}

template <typename F, int PL, bool J64L>
__global__ __launch_bounds__(2 * kMaxSweepThreads) void k_refresh(Inst P, LdsPlan plan)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int w = blockIdx.x;
    Walker<F> W = carve<F, PL, J64L>(lds, plan, P, w);
    load_walker<F>(P, W, plan, w);
    const double E = refresh_fields<F>(P, W);
    __syncthreads();
    store_walker<F>(P, W, plan, w);
    if (threadIdx.x == 0) {
        P.E[w] = E;
        P.Eerr[w] = P.ebound;
        P.nupd[w] = 0;
        int nmax = 0;
        for (int k = 0; k < P.q; ++k) nmax = max(nmax, W.cnt[k]);
        P.Mw[w] = (static_cast<double>(P.q) * nmax / P.L - 1.0) / (P.q - 1);
    }
}

// The life of one walker of instance P through sweeps n0 .. n0 + nsw - 1:
// load its state into LDS, sweep, record, refresh on schedule, and (fused)
// meet the instance's other walkers at the device barrier for the exchange.
// Returns false if the barrier timed out.
template <typename F, int QT, int PL, bool J64L, bool OV = false>
__device__ __forceinline__ bool run_walker(const Inst &P, const LdsPlan &plan, unsigned char *lds, int w, int64_t n0,
                                           int32_t nsw, int32_t xevery, int32_t x0, int64_t m0, bool fused)
{
    const int tid = threadIdx.x;
    PhaseAcc ph;
    // thread 0 keeps the phases; in an overlapped sweep the flush waves' first
    // thread keeps the flush's own cycles
    ph.on = P.phase != nullptr && (tid == 0 || (OV && tid == static_cast<int>(blockDim.x) / 2));
    for (int k = 0; k < kPhN; ++k) ph.v[k] = 0;
    const uint64_t t_begin = ph.on ? clock64() : 0;
    constexpr bool TAB = PL != kPlDirect;
    constexpr bool kF32Tab = TAB && table_prec<F>() == kPrecF32;
    Walker<F> W = carve<F, PL, J64L>(lds, plan, P, w);
    load_walker<F>(P, W, plan, w);
    ChainRegs cr{P.E[w], P.Eerr[w], P.nupd[w], 0, 0.0, 0.0, 0u};
    int64_t m = m0;
    __syncthreads();
    for (int s = 0; s < nsw; ++s) {
        const int64_t n = n0 + s;
        const int slot = __hip_atomic_load(&P.slot_of[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double beta = P.beta[slot];
        cr.nacc = 0;
        double part;
        if constexpr (OV)
            part = sweep_walker_ov<F, QT>(P, W, w, n, beta, cr, ph);
        else
            part = sweep_walker<F, QT, PL>(P, W, w, n, beta, cr, ph);
        ph_start(ph);
        // energy change of the sweep: the flush's sums over the FP32 couplings
        // (FP32 table) or the accepted flips' dE held by the chain lanes (FP64
        // table, or direct sums when there is no table)
        cr.E += block_sum(part + cr.eL, W.red) * P.qscale;
        cr.Eerr += block_sum(cr.errL, W.red) * P.qscale;
        cr.eL = cr.errL = 0.0;
        if (tid == 0) {
            W.cs->nupd = cr.nupd;
            W.cs->nacc = cr.nacc;
        }
        __syncthreads();
        cr.nupd = W.cs->nupd;
        cr.nacc = W.cs->nacc;
        if (kF32Tab) cr.Eerr += static_cast<double>(cr.nacc) * P.bound_flipE;
        record_sweep<F>(P, W, w, slot, n, cr.E, cr.nacc);
        // without a table there is nothing to refresh (energies come from direct sums)
        if (TAB && ((P.refresh_every > 0 && (n + 1) % P.refresh_every == 0) || cr.nupd > P.nupd_max)) {
            cr.E = refresh_fields<F>(P, W);
            cr.Eerr = P.ebound;
            cr.nupd = 0;
            if (tid == 0) atomicAdd(&P.ctr[kCtrRefresh], 1ull);
            __syncthreads();
        }
        ph_mark(ph, kPhRecord);
        // x0: sweeps of the same exchange period done before this launch
        if (fused && xevery > 0 && (x0 + s + 1) % xevery == 0) {
            for (int j = tid; j < P.L; j += blockDim.x) P.spins[static_cast<size_t>(w) * P.L + j] = W.sp[j];
            if (tid == 0) {
                P.E[w] = cr.E;
                P.Eerr[w] = cr.Eerr;
            }
            if (grid_arrive(P, W.misc)) {
                exchange_step(P, m, carve_x(lds + plan.xch, P.R), W.red);
                grid_release(P, W.misc);
            } else if (!grid_wait(P, W.misc)) {
                return false;  // time-out or error raised elsewhere: leave; the host reports it
            }
            cr.E = __hip_atomic_load(&P.E[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cr.Eerr = __hip_atomic_load(&P.Eerr[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++m;
            ph_mark(ph, kPhExchange);
        }
    }
    __syncthreads();
    store_walker<F>(P, W, plan, w);
    if (tid == 0) {
        P.E[w] = cr.E;
        P.Eerr[w] = cr.Eerr;
        P.nupd[w] = cr.nupd;
    }
    if (ph.on) {
        unsigned long long *dst = P.phase + static_cast<size_t>(w) * kPhN;
        if (tid == 0) {
            ph.v[kPhTotal] = clock64() - t_begin;
            ph.v[kPhIters] = cr.iters;
            for (int k = 0; k < kPhN; ++k) atomicAdd(&dst[k], ph.v[k]);
        } else {  // the flush waves' counter (overlapped sweep)
            atomicAdd(&dst[kPhFlush], ph.v[kPhFlush]);
            atomicAdd(&dst[kPhFlushes], ph.v[kPhFlushes]);
        }
    }
    __syncthreads();
    return true;
}

template <typename F, int QT, int PL, bool J64L, bool OV = false>
__global__ __launch_bounds__(OV ? 2 * kMaxSweepThreads : kMaxSweepThreads) void k_sweep(
    Inst P, LdsPlan plan, int64_t n0, int32_t nsw, int32_t xevery, int32_t x0, int64_t m0, int32_t fused)
{
    extern __shared__ __align__(16) unsigned char lds[];
    (void)run_walker<F, QT, PL, J64L, OV>(P, plan, lds, blockIdx.x, n0, nsw, xevery, x0, m0, fused != 0);
}

static __global__ __launch_bounds__(1024) void k_exchange(Inst P, int64_t m)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double *red = reinterpret_cast<double *>(lds);
    exchange_step(P, m, carve_x(lds + 256, P.R), red);
}

}  // namespace ptmi

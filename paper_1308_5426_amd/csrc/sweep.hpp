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
// One workgroup owns one walker (replica).  Every wave of the workgroup
// evaluates the same window of 64 consecutive attempts (lane = attempt), so
// all waves take identical decisions without communicating; the first lane
// that is accepted (or needs an FP64 recheck) is applied, the earlier lanes
// were rejections and changed nothing, and the window continues after it.
// This "lookahead" keeps the sequential semantics of the Markov chain exact.
#pragma once
#include "device_common.hpp"
#include "state.hpp"

namespace ptmi {

// LDS carve (byte offsets), computed on the host by lds_plan().
struct LdsPlan {
    int32_t J, h, J64, masks, sp, cnt, red, misc, xch, total;
    int32_t j64_in_lds;   // 1: FP64 couplings resident in LDS
    int32_t h_in_lds;     // 1: field table in LDS; 0: the walker's rows stay in HBM
};

// Margin for the FP64 evaluation of beta dE + ln u beyond the table bound
// (FP64 rounding of the products and of the library logarithm).
constexpr double kEvalMargin = 1e-12;
// Grid barrier time-out, in wall-clock ticks (100 MHz on gfx9): 20 s.
constexpr uint64_t kBarrierTicks = 2000000000ull;

template <typename F>
struct Walker {
    F *J;               // [L] couplings in the table's precision
    F *h;               // [q][L] field table
    const double *J64;  // [L] FP64 couplings (LDS or HBM)
    uint8_t *sp;        // [L] spins 0..q-1
    int32_t *cnt;       // [kQMax]
    uint64_t *masks;    // [q][ceil(L/64)] sites per state, for the refresh
    double *red;        // [16] reduction scratch
    int32_t *misc;      // [8]
};

template <typename F>
__device__ __forceinline__ Walker<F> carve(unsigned char *lds, const LdsPlan &p, const Inst &P, int w)
{
    Walker<F> W;
    W.J = reinterpret_cast<F *>(lds + p.J);
    W.h = p.h_in_lds ? reinterpret_cast<F *>(lds + p.h)
                     : static_cast<F *>(P.h) + static_cast<size_t>(w) * P.q * P.L;
    W.J64 = p.j64_in_lds ? reinterpret_cast<const double *>(lds + p.J64) : P.J64;
    W.sp = lds + p.sp;
    W.cnt = reinterpret_cast<int32_t *>(lds + p.cnt);
    W.masks = reinterpret_cast<uint64_t *>(lds + p.masks);
    W.red = reinterpret_cast<double *>(lds + p.red);
    W.misc = reinterpret_cast<int32_t *>(lds + p.misc);
    return W;
}

template <typename F>
__device__ __forceinline__ const F *coupling_src(const Inst &P);
template <>
__device__ __forceinline__ const float *coupling_src<float>(const Inst &P) { return P.J32; }
template <>
__device__ __forceinline__ const double *coupling_src<double>(const Inst &P) { return P.J64; }

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
__global__ void k_init_spins(Inst P, int32_t ordered)
{
    const int64_t total = static_cast<int64_t>(P.R) * P.L;
    for (int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int w = static_cast<int>(e / P.L), j = static_cast<int>(e % P.L);
        uint8_t v = 0;
        if (!ordered) {
            const uint4 o = philox10(make_uint4(static_cast<uint32_t>(j), 0u, static_cast<uint32_t>(w), 2u),
                                     P.key0, P.key1);
            v = static_cast<uint8_t>(__umulhi(o.x, static_cast<uint32_t>(P.q)));
        }
        P.spins[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Walker state HBM <-> LDS.
// ---------------------------------------------------------------------------
template <typename F>
__device__ void load_walker(const Inst &P, Walker<F> &W, const LdsPlan &plan, int w)
{
    const int L = P.L, q = P.q;
    const F *Jsrc = coupling_src<F>(P);
    const F *hsrc = static_cast<const F *>(P.h) + static_cast<size_t>(w) * q * L;
    const uint8_t *ssrc = P.spins + static_cast<size_t>(w) * L;
    double *J64l = plan.j64_in_lds && sizeof(F) != sizeof(double) ? const_cast<double *>(W.J64) : nullptr;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        W.J[j] = Jsrc[j];
        W.sp[j] = ssrc[j];
        if (J64l) J64l[j] = P.J64[j];
    }
    if (plan.h_in_lds)
        for (int e = threadIdx.x; e < q * L; e += blockDim.x) W.h[e] = hsrc[e];
    if (threadIdx.x < kQMax) W.cnt[threadIdx.x] = P.counts[w * kQMax + threadIdx.x];
}

template <typename F>
__device__ void store_walker(const Inst &P, const Walker<F> &W, const LdsPlan &plan, int w)
{
    const int L = P.L, q = P.q;
    F *hdst = static_cast<F *>(P.h) + static_cast<size_t>(w) * q * L;
    uint8_t *sdst = P.spins + static_cast<size_t>(w) * L;
    for (int j = threadIdx.x; j < L; j += blockDim.x) sdst[j] = W.sp[j];
    if (plan.h_in_lds)
        for (int e = threadIdx.x; e < q * L; e += blockDim.x) hdst[e] = W.h[e];
    if (threadIdx.x < kQMax) P.counts[w * kQMax + threadIdx.x] = W.cnt[threadIdx.x];
}

// ---------------------------------------------------------------------------
// Field table from the spins, FP64 accumulation.  For each state k a bitmask
// per 64-site block lists the sites in state k; every thread owns sites j
// and walks the set bits (wave-uniform, scalar), adding J*(|j - i|).  The
// energy E = -1/2 sum_j h[s_j][j] is formed from the FP64 sums.
// ---------------------------------------------------------------------------
template <typename F>
__device__ double refresh_fields(const Inst &P, Walker<F> &W)
{
    const int L = P.L, q = P.q, tid = threadIdx.x, NT = blockDim.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave, nw = NT / kWave;
    const int nblk = (L + kWave - 1) / kWave;
    __syncthreads();
    for (int blk = wv; blk < nblk; blk += nw) {
        const int j = blk * kWave + lane;
        const int s = j < L ? W.sp[j] : -1;
        for (int k = 0; k < q; ++k) {
            const uint64_t m = __ballot(s == k);
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
                    acc += W.J64[d];  // J*(0) = 0 removes the self term
                }
            }
            if (ok) {
                W.h[k * L + j] = static_cast<F>(acc);
                if (k == sj) epart += acc;
            }
        }
    }
    return -0.5 * block_sum(epart, W.red);
}

// dE = sum_{j != i} J*(|i-j|) [delta(a, s_j) - delta(b, s_j)] in FP64 (the
// plain definition), reduced over the workgroup in a fixed order.
template <typename F>
__device__ double direct_dE(const Walker<F> &W, int L, int i, int a, int b)
{
    double part = 0.0;
    for (int j = threadIdx.x; j < L; j += blockDim.x) {
        const int s = W.sp[j];
        int d = j - i;
        d += d < 0 ? L : 0;
        const double jv = W.J64[d];
        part += s == a ? jv : (s == b ? -jv : 0.0);
    }
    return block_sum(part, W.red);
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
        }
        __syncthreads();
        for (int p = 0; p < npair; ++p) {  // rare: uncertain pairs, whole workgroup
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
            P.xatt[k] += 1;
            if (acc) {
                X.perm[k] = wb;
                X.perm[k + 1] = wa;
                P.xacc[k] += 1;
            }
        }
        __syncthreads();
    }
    for (int k = tid; k < R; k += NT) {
        P.perm[k] = X.perm[k];
        P.slot_of[X.perm[k]] = k;
        P.E[k] = X.E[k];
        P.Eerr[k] = X.Eerr[k];
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

__device__ bool grid_arrive(const Inst &P, int32_t *flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned g = __hip_atomic_load(bar_gen(P), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned old = __hip_atomic_fetch_add(bar_count(P), 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        flag[0] = old == gridDim.x - 1;
        flag[1] = static_cast<int32_t>(g);
        if (flag[0]) __threadfence();
    }
    __syncthreads();
    return flag[0] != 0;
}

__device__ void grid_release(const Inst &P, int32_t *flag)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
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
        __threadfence();
        flag[2] = ok;
    }
    __syncthreads();
    return flag[2] != 0;
}

// ---------------------------------------------------------------------------
// One sweep of L attempts of walker w at sweep index n (counter (t, n, w, 0)).
// ---------------------------------------------------------------------------
template <typename F>
__device__ void metropolis_sweep(const Inst &P, Walker<F> &W, int w, int64_t n, double beta, double &E,
                                 double &Eerr, int64_t &nupd, int64_t &nacc)
{
    const int L = P.L, q = P.q, tid = threadIdx.x, NT = blockDim.x, lane = tid & (kWave - 1);
    for (int t0 = 0; t0 < L; t0 += kWave) {
        const int ta = t0 + lane;
        const uint4 o = philox10(make_uint4(static_cast<uint32_t>(ta), static_cast<uint32_t>(n),
                                            static_cast<uint32_t>(w), 0u),
                                 P.key0, P.key1);
        const int i = static_cast<int>(__umulhi(o.x, static_cast<uint32_t>(L)));
        const int kk = 1 + static_cast<int>(__umulhi(o.y, static_cast<uint32_t>(q - 1)));
        const double lnu = log(open_unit(o.z, o.w));
        uint64_t live = __ballot(ta < L);
        while (live) {
            const int a = W.sp[i];
            int b = a + kk;
            b -= b >= q ? q : 0;
            const double dE = static_cast<double>(W.h[a * L + i]) - static_cast<double>(W.h[b * L + i]);
            const double x = beta * dE + lnu;
            const double Bd = 2.0 * (P.bound_init + static_cast<double>(nupd) * P.bound_unit);
            const double trig = beta * Bd + kBand + kEvalMargin;
            const uint64_t cand = __ballot(x < trig) & live;
            if (cand == 0) break;
            const int f = __ffsll(static_cast<unsigned long long>(cand)) - 1;
            const int i_f = __shfl(i, f), a_f = __shfl(a, f), b_f = __shfl(b, f);
            const double x_f = __shfl(x, f), lnu_f = __shfl(lnu, f), dE_f = __shfl(dE, f);
            bool accept = true;
            double dEuse = dE_f, errinc = Bd;
            if (!(x_f < -trig)) {
                // |x| within the trigger band: decide with the FP64 direct sum
                const double d64 = direct_dE(W, L, i_f, a_f, b_f);
                const double x64 = beta * d64 + lnu_f;
                accept = x64 < 0.0;
                dEuse = d64;
                errinc = 0.0;
                if (tid == 0) {
                    atomicAdd(&P.ctr[kCtrRecheck], 1ull);
                    if (fabs(x64) <= kBand) {
                        atomicAdd(&P.ctr[kCtrBandedMet], 1ull);
                        log_event(P, 0, w, n, t0 + f, accept ? 1 : 0, x64);
                    }
                }
            }
            if (accept) {
                __syncthreads();  // every wave has read the table for this window
                F *ha = W.h + a_f * L;
                F *hb = W.h + b_f * L;
                for (int j = tid; j < L; j += NT) {
                    int d = j - i_f;
                    d += d < 0 ? L : 0;
                    const F jv = W.J[d];
                    ha[j] -= jv;
                    hb[j] += jv;
                }
                if (tid == 0) {
                    W.sp[i_f] = static_cast<uint8_t>(b_f);
                    W.cnt[a_f] -= 1;
                    W.cnt[b_f] += 1;
                }
                E += dEuse;
                Eerr += errinc;
                ++nupd;
                ++nacc;
                __syncthreads();
            }
            live &= f == kWave - 1 ? 0ull : (~0ull << (f + 1));
        }
    }
}

template <typename F>
__device__ void record_sweep(const Inst &P, const Walker<F> &W, int w, int slot, int64_t n, double E, int64_t nacc)
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
template <typename F>
__global__ __launch_bounds__(1024) void k_refresh(Inst P, LdsPlan plan)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int w = blockIdx.x;
    Walker<F> W = carve<F>(lds, plan, P, w);
    load_walker<F>(P, W, plan, w);
    const double E = refresh_fields<F>(P, W);
    __syncthreads();
    store_walker<F>(P, W, plan, w);
    if (threadIdx.x == 0) {
        P.E[w] = E;
        P.Eerr[w] = 0.0;
        P.nupd[w] = 0;
        int nmax = 0;
        for (int k = 0; k < P.q; ++k) nmax = max(nmax, W.cnt[k]);
        P.Mw[w] = (static_cast<double>(P.q) * nmax / P.L - 1.0) / (P.q - 1);
    }
}

template <typename F>
__global__ __launch_bounds__(1024) void k_sweep(Inst P, LdsPlan plan, int64_t n0, int32_t nsw, int32_t xevery,
                                                int64_t m0, int32_t fused)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int w = blockIdx.x, tid = threadIdx.x;
    Walker<F> W = carve<F>(lds, plan, P, w);
    load_walker<F>(P, W, plan, w);
    double E = P.E[w], Eerr = P.Eerr[w];
    int64_t nupd = P.nupd[w];
    int64_t m = m0;
    __syncthreads();
    for (int s = 0; s < nsw; ++s) {
        const int64_t n = n0 + s;
        const int slot = __hip_atomic_load(&P.slot_of[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double beta = P.beta[slot];
        int64_t nacc = 0;
        metropolis_sweep<F>(P, W, w, n, beta, E, Eerr, nupd, nacc);
        __syncthreads();
        record_sweep<F>(P, W, w, slot, n, E, nacc);
        if ((P.refresh_every > 0 && (n + 1) % P.refresh_every == 0) || nupd > P.nupd_max) {
            E = refresh_fields<F>(P, W);
            Eerr = 0.0;
            nupd = 0;
            if (tid == 0) atomicAdd(&P.ctr[kCtrRefresh], 1ull);
            __syncthreads();
        }
        if (fused && xevery > 0 && (s + 1) % xevery == 0) {
            for (int j = tid; j < P.L; j += blockDim.x) P.spins[static_cast<size_t>(w) * P.L + j] = W.sp[j];
            if (tid == 0) {
                P.E[w] = E;
                P.Eerr[w] = Eerr;
            }
            if (grid_arrive(P, W.misc)) {
                exchange_step(P, m, carve_x(lds + plan.xch, P.R), W.red);
                grid_release(P, W.misc);
            } else if (!grid_wait(P, W.misc)) {
                return;  // time-out or error raised elsewhere: leave; the host reports it
            }
            E = __hip_atomic_load(&P.E[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            Eerr = __hip_atomic_load(&P.Eerr[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ++m;
        }
    }
    __syncthreads();
    store_walker<F>(P, W, plan, w);
    if (tid == 0) {
        P.E[w] = E;
        P.Eerr[w] = Eerr;
        P.nupd[w] = nupd;
    }
}

__global__ __launch_bounds__(1024) void k_exchange(Inst P, int64_t m)
{
    extern __shared__ __align__(16) unsigned char lds[];
    double *red = reinterpret_cast<double *>(lds);
    exchange_step(P, m, carve_x(lds + 256, P.R), red);
}

}  // namespace ptmi

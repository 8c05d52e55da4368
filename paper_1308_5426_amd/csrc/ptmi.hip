// ptmi.hip -- host runtime and C ABI of the gfx950 parallel-tempering library
// for the 1D long-range q-state Potts ring (see include/ptmi.h for the
// contract of every entry point and the paper passages they implement).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ptmi.h"
#include "kernels.hpp"

using namespace ptmi;

static_assert(sizeof(pt_event) == sizeof(Event), "event layout");
static_assert(PT_QMAX == kQMax, "q limit");

namespace {

// A fixed buffer, so that reporting an error allocates nothing either.
thread_local char g_err[512];

pt_status fail(pt_status st, const char *fmt, ...)
{
    char buf[sizeof g_err];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::memcpy(g_err, buf, sizeof buf);
    return st;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(PT_EDEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                                          __FILE__, __LINE__);                                    \
    } while (0)

constexpr uint32_t kMagic = 0x50544d49u;  // "PTMI"
constexpr uint32_t kVersion = 1;

}  // namespace

struct pt_ctx {
    int32_t L = 0, q = 0, R = 0, prec = 0, init = 0, NT = 64, refresh_every = 0, ser_cap = 0,
            ev_cap = 0, max_chunk = 0, device = 0, cus = 0;
    double sigma = 0.0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    unsigned char *ws = nullptr;
    size_t ws_bytes = 0;
    bool own_ws = false;
    bool failed = false;
    Inst inst{};
    LdsPlan plan{}, plan_fused{};
    bool can_fuse = false;
    bool h_in_lds = true;
    bool prof = false;
    int64_t sweeps = 0, xsteps = 0, samples = 0;
    std::vector<double> T;
};

namespace {

size_t field_bytes(int prec) { return prec == PT_PREC_F64 ? sizeof(double) : 4; }

bool valid_prec(int prec) { return prec == PT_PREC_F64 || prec == PT_PREC_F32 || prec == PT_PREC_I32; }

// One wave per 256 sites, up to one wave per SIMD.
int auto_threads(int L)
{
    const int waves = std::min(kMaxSweepThreads / kWave, std::max(1, (L + 255) / 256));
    return waves * kWave;
}

int32_t align16(int32_t x) { return (x + 15) & ~15; }

bool make_plan_chunk(int L, int q, int R, int prec, bool fused, int place, size_t lds_max, int chunk,
                     int threads, LdsPlan *p, bool ovl)
{
    const bool h_in_lds = place == kPlLds;
    p->place = place;
    p->ovl = ovl ? 1 : 0;
    const int32_t fb = static_cast<int32_t>(field_bytes(prec));
    const int nblk = (L + kWave - 1) / kWave;
    // the waves that run the chain (overlapped: half of them) and the threads that flush
    const int nw = threads / kWave / (ovl ? 2 : 1);
    const int flush_threads = ovl ? threads / 2 : threads;
    // with the table in LDS the coupling row is doubled and padded to the
    // flush's site slots: J[k] = J*(k mod L) for k < L + passes * threads * kFlushM
    const int span = flush_threads * kFlushM;
    p->jlen = h_in_lds ? L + (L + span - 1) / span * span : L;
    int32_t o = 0;
    p->J = o; o = align16(o + fb * p->jlen);
    p->h_in_lds = h_in_lds ? 1 : 0;
    p->h = o;
    if (h_in_lds) o = align16(o + fb * (q - 1) * L);  // row q-1 is implicit
    p->sp = o; o = align16(o + L);
    p->cnt = o; o = align16(o + 4 * kQMax);
    p->red = o; o = align16(o + 8 * 32);
    p->misc = o; o = align16(o + 4 * 8);
    p->pend = o; o = align16(o + 2 * 4 * kWave);  // two flip lists (overlapped sweep: by window parity)
    p->cs = o; o = align16(o + static_cast<int32_t>(sizeof(ChainState)));
    p->ctab = o; o = align16(o + 256 * fb);
    // one scratch region for three uses that never overlap in time: the
    // refresh's per-state site masks, the exchange step's scratch, and the
    // sweep's staging (draws, ln u, the waves' partial corrections)
    p->chunk = chunk;
    const int32_t sweep_bytes = align16(4 * chunk) + align16(8 * chunk) + align16(2 * nw * kWave * 8);
    const int32_t scratch = std::max({align16(8 * q * nblk), fused ? align16(40 * R) : 0, sweep_bytes});
    p->masks = o;
    p->xch = o;
    p->draw = o;
    p->dlnu = p->draw + align16(4 * chunk);
    p->xpart = p->dlnu + align16(8 * chunk);
    o += scratch;
    if (prec == PT_PREC_F64) {
        p->J64 = p->J;
        p->j64_in_lds = 1;
    } else if (prec == PT_PREC_F32 && static_cast<size_t>(o) + 8u * L <= lds_max) {
        // (int tables recheck rarely: their FP64 couplings stay in HBM)
        p->J64 = o;
        o = align16(o + 8 * L);
        p->j64_in_lds = 1;
    } else {
        p->J64 = 0;
        p->j64_in_lds = 0;
    }
    // optional: the chain's first-guessed-flip tables (4 B per site and wave)
    if (static_cast<size_t>(o) + 4u * L * nw <= lds_max) {
        p->sfirst = o;
        o = align16(o + 4 * L * nw);
    } else {
        p->sfirst = -1;
    }
    p->total = o;
    return static_cast<size_t>(o) <= lds_max;
}

// LDS carve: couplings, field table, spins, counts, reduction scratch, flags,
// pending flips, flush coefficients, one shared scratch region (refresh
// masks / exchange scratch / staged draws of the largest chunk of 64..1024
// attempts that fits), FP64 couplings and the first-guessed-flip tables when
// they fit.
bool make_plan(int L, int q, int R, int prec, bool fused, int place, size_t lds_max, int threads, LdsPlan *p,
               bool ovl = false)
{
    const int lmax = std::min(1024, ((L + kWave - 1) / kWave) * kWave);
    if (make_plan_chunk(L, q, R, prec, fused, place, lds_max, lmax, threads, p, ovl)) return true;
    if (ovl) return false;  // the overlapped sweep stages a whole sweep's draws
    for (int chunk = 512; chunk >= kWave; chunk /= 2)
        if (chunk < lmax && make_plan_chunk(L, q, R, prec, fused, place, lds_max, chunk, threads, p, false)) return true;
    return false;
}

Layout layout_of(int L, int q, int R, int prec, int ser_cap, int ev_cap, bool prof = false)
{
    return Layout(L, q, R, field_bytes(prec), ser_cap, ev_cap, prof);
}

pt_status validate(int32_t L, int32_t q, double sigma, const double *T, int32_t R)
{
    if (L < 2 || L > 65535) return fail(PT_EINVAL, "L must be in [2, 65535] (got %d)", L);
    if (q < 2 || q > PT_QMAX) return fail(PT_EINVAL, "q must be in [2, %d] (got %d)", PT_QMAX, q);
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(PT_EINVAL, "sigma must be finite and > 0");
    if (R < 1) return fail(PT_EINVAL, "R must be >= 1");
    if (!T) return fail(PT_EINVAL, "T is NULL");
    for (int k = 0; k < R; ++k) {
        if (!(T[k] > 0.0) || !std::isfinite(T[k])) return fail(PT_EINVAL, "T[%d] must be finite and > 0", k);
        if (k > 0 && T[k] < T[k - 1]) return fail(PT_EINVAL, "T must be ascending (T[%d] < T[%d])", k, k - 1);
    }
    return PT_OK;
}

// Kernels by table precision (each precision's kernels are built in a source
// file of their own, kernels_<prec>.hip).
const void *sweep_fn_prec(int prec, int q, const LdsPlan &p)
{
    if (prec == PT_PREC_F32) return sweep_kernel_f32(q, p);
    if (prec == PT_PREC_I32) return sweep_kernel_i32(q, p);
    return sweep_kernel_f64(q, p);
}
const void *refresh_fn_prec(int prec, const LdsPlan &p)
{
    if (prec == PT_PREC_F32) return refresh_kernel_f32(p);
    if (prec == PT_PREC_I32) return refresh_kernel_i32(p);
    return refresh_kernel_f64(p);
}

pt_status set_lds_attr(const void *fn, int bytes)
{
    HIPCHK(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    return PT_OK;
}

pt_status launch_refresh(pt_ctx *c)
{
    Inst P = c->inst;
    LdsPlan plan = c->plan;
    void *args[] = {&P, &plan};
    HIPCHK(hipLaunchKernel(refresh_fn_prec(c->prec, plan), dim3(c->R), dim3(c->NT), args, plan.total, c->stream));
    return PT_OK;
}

pt_status launch_sweep(pt_ctx *c, int64_t n0, int32_t nsw, int32_t xevery, int32_t x0, int64_t m0, bool fused)
{
    Inst P = c->inst;
    LdsPlan plan = fused ? c->plan_fused : c->plan;
    int32_t fu = fused ? 1 : 0;
    void *args[] = {&P, &plan, &n0, &nsw, &xevery, &x0, &m0, &fu};
    const void *fn = sweep_fn_prec(c->prec, c->q, plan);
    if (fused)
        HIPCHK(hipLaunchCooperativeKernel(fn, dim3(c->R), dim3(c->NT), args, plan.total, c->stream));
    else
        HIPCHK(hipLaunchKernel(fn, dim3(c->R), dim3(c->NT), args, plan.total, c->stream));
    return PT_OK;
}

pt_status launch_exchange(pt_ctx *c)
{
    const int bytes = 256 + 40 * c->R;
    hipLaunchKernelGGL(k_exchange, dim3(1), dim3(std::min(1024, std::max(64, ((c->R + 63) / 64) * 64))),
                       bytes, c->stream, c->inst, c->xsteps);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

// Queues a zero fill of n bytes at p on stream st.
pt_status zero_async(void *p, size_t n, hipStream_t st)
{
    if (n == 0) return PT_OK;
    const size_t words = (n + 7) / 8;
    const unsigned blocks = static_cast<unsigned>(std::min<size_t>(2048, (words + 255) / 256));
    hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, static_cast<unsigned char *>(p), n);
    HIPCHK(hipGetLastError());
    return PT_OK;
}

pt_status check_ctx(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    if (c->failed) return fail(PT_ESTATE, "context is in a failed state");
    return PT_OK;
}

pt_status device_error(pt_ctx *c)
{
    unsigned long long err = 0;
    HIPCHK(hipMemcpy(&err, c->inst.ctr + kCtrError, sizeof err, hipMemcpyDeviceToHost));
    if (err) {
        c->failed = true;
        return fail(PT_EDEVICE, "kernel reported error bits 0x%llx (grid barrier time-out)", err);
    }
    return PT_OK;
}

// Points an instance's arrays into its workspace block.
void fill_inst(Inst &P, unsigned char *b, const Layout &lay, int L, int q, int R, uint64_t seed, int refresh_every,
               int ser_cap, int ev_cap, bool prof = false)
{
    P = Inst{};
    P.L = L; P.q = q; P.R = R; P.walker0 = 0;
    P.key0 = static_cast<uint32_t>(seed);
    P.key1 = static_cast<uint32_t>(seed >> 32);
    P.refresh_every = refresh_every;
    P.ser_cap = ser_cap;
    P.J64 = reinterpret_cast<const double *>(b + lay.J64);
    P.J32 = reinterpret_cast<const float *>(b + lay.J32);
    P.Jq = reinterpret_cast<const int32_t *>(b + lay.Jq);
    P.spins = b + lay.spins;
    P.h = b + lay.h;
    P.E = reinterpret_cast<double *>(b + lay.E);
    P.Eerr = reinterpret_cast<double *>(b + lay.Eerr);
    P.nupd = reinterpret_cast<int64_t *>(b + lay.nupd);
    P.counts = reinterpret_cast<int32_t *>(b + lay.counts);
    P.Mw = reinterpret_cast<double *>(b + lay.Mw);
    P.perm = reinterpret_cast<int32_t *>(b + lay.perm);
    P.slot_of = reinterpret_cast<int32_t *>(b + lay.slot_of);
    P.beta = reinterpret_cast<const double *>(b + lay.beta);
    P.acc6 = reinterpret_cast<double *>(b + lay.acc6);
    P.fatt = reinterpret_cast<int64_t *>(b + lay.fatt);
    P.facc = reinterpret_cast<int64_t *>(b + lay.facc);
    P.xatt = reinterpret_cast<int64_t *>(b + lay.xatt);
    P.xacc = reinterpret_cast<int64_t *>(b + lay.xacc);
    P.serE = reinterpret_cast<double *>(b + lay.serE);
    P.serM = reinterpret_cast<double *>(b + lay.serM);
    P.events = reinterpret_cast<Event *>(b + lay.events);
    P.ev_cap = ev_cap;
    P.ctr = reinterpret_cast<unsigned long long *>(b + lay.ctr);
    P.bnd = reinterpret_cast<TableBounds *>(b + lay.bnd);
    P.phase = prof ? reinterpret_cast<unsigned long long *>(b + lay.phase) : nullptr;
}

// Host copy of an instance's observables (by walker / slot as on the device).
struct HostObs {
    int R = 0, q = 0, L = 0;
    std::vector<double> Ew, Mw, acc6;
    std::vector<int32_t> perm;
    std::vector<int64_t> fatt, facc, xatt, xacc;
    std::vector<unsigned long long> ctr;
    int ev_cap = 0;

    pt_status fetch(const Inst &P, hipStream_t st)
    {
        R = P.R; q = P.q; L = P.L; ev_cap = P.ev_cap;
        Ew.resize(R); Mw.resize(R); acc6.resize(6 * R); perm.resize(R);
        fatt.resize(R); facc.resize(R); xatt.resize(R); xacc.resize(R); ctr.resize(kCtrN);
        HIPCHK(hipMemcpyAsync(Ew.data(), P.E, sizeof(double) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(Mw.data(), P.Mw, sizeof(double) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(acc6.data(), P.acc6, sizeof(double) * 6 * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(perm.data(), P.perm, sizeof(int32_t) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(fatt.data(), P.fatt, sizeof(int64_t) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(facc.data(), P.facc, sizeof(int64_t) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(xatt.data(), P.xatt, sizeof(int64_t) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(xacc.data(), P.xacc, sizeof(int64_t) * R, hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(ctr.data(), P.ctr, sizeof(unsigned long long) * kCtrN, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return PT_OK;
    }

    void fill(pt_obs *o, int64_t sweeps, int64_t xsteps, int64_t samples) const
    {
        o->R = R; o->q = q; o->L = L;
        o->sweeps = sweeps; o->exchange_steps = xsteps; o->samples = samples;
        for (int k = 0; k < R; ++k) {
            if (o->E) o->E[k] = Ew[perm[k]];
            if (o->M) o->M[k] = Mw[perm[k]];
            double *dst[6] = {o->sumE, o->sumE2, o->sumE4, o->sumM, o->sumM2, o->sumM4};
            for (int a = 0; a < 6; ++a)
                if (dst[a]) dst[a][k] = acc6[a * R + k];
            if (o->flip_att) o->flip_att[k] = fatt[k];
            if (o->flip_acc) o->flip_acc[k] = facc[k];
            if (o->perm) o->perm[k] = perm[k];
            if (k + 1 < R) {
                if (o->xchg_att) o->xchg_att[k] = xatt[k];
                if (o->xchg_acc) o->xchg_acc[k] = xacc[k];
            }
        }
        o->n_recheck = static_cast<int64_t>(ctr[kCtrRecheck]);
        o->n_banded = static_cast<int64_t>(ctr[kCtrBandedMet] + ctr[kCtrBandedEx]);
        o->n_exact_energy = static_cast<int64_t>(ctr[kCtrExactE]);
        o->n_refresh = static_cast<int64_t>(ctr[kCtrRefresh]);
        o->n_events_dropped = ctr[kCtrEvents] > static_cast<unsigned long long>(ev_cap)
                                  ? static_cast<int64_t>(ctr[kCtrEvents] - ev_cap)
                                  : 0;
    }
};

// Ladder, slot permutation and table bounds of a fresh instance on the device
// (k_setup, after k_jstar), then the bounds read back into the instance
// parameters.  T is copied into the instance's workspace first.  Synchronises
// the stream.  Allocates nothing.
pt_status setup_instance(pt_ctx *c, const double *T)
{
    Inst &P = c->inst;
    const Layout lay = layout_of(c->L, c->q, c->R, c->prec, c->ser_cap, c->ev_cap, c->prof);
    double *Td = reinterpret_cast<double *>(c->ws + lay.T);
    HIPCHK(hipMemcpyAsync(Td, T, sizeof(double) * c->R, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_setup, dim3(1), dim3(256), 0, c->stream, P, static_cast<const double *>(Td),
                       static_cast<int32_t>(c->prec));
    HIPCHK(hipGetLastError());
    TableBounds b;
    HIPCHK(hipMemcpyAsync(&b, P.bnd, sizeof b, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    // J*(r) > 0 for every r, so a finite sum means finite couplings
    if (!std::isfinite(b.init) || !std::isfinite(b.unit) || !(b.init > 0.0))
        return fail(PT_EDEVICE, "non-finite couplings J* (L = %d, sigma = %g)", c->L, c->sigma);
    P.bound_init = b.init;
    P.bound_unit = b.unit;
    P.nupd_max = b.nupd_max;
    P.bound_flipE = b.flipE;
    P.ebound = b.ebound;
    P.qscale = b.qscale;
    P.hsum = b.hsum;
    P.bound_rows = b.rows;
    P.bound_impl = b.impl;
    return PT_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void pt_default_options(pt_options *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->precision = PT_PREC_F64;
    o->init = PT_INIT_RANDOM;
    o->placement = PT_PLACE_AUTO;
}

const char *pt_last_error(void) { return g_err; }

pt_status pt_workspace_size(int32_t L, int32_t q, int32_t R, const pt_options *opt, size_t *bytes)
{
    if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
    if (L < 2 || q < 2 || q > PT_QMAX || R < 1) return fail(PT_EINVAL, "bad sizes");
    pt_options d;
    pt_default_options(&d);
    const pt_options &o = opt ? *opt : d;
    const int ev = o.event_capacity > 0 ? o.event_capacity : 4096;
    *bytes = layout_of(L, q, R, o.precision, std::max(0, o.series_capacity), ev, o.profile != 0).total;
    return PT_OK;
}

// Checks the options of a single instance.
static pt_status check_options(const pt_options &o)
{
    if (!valid_prec(o.precision)) return fail(PT_EINVAL, "bad precision");
    if (o.precision == PT_PREC_I32 && o.placement == PT_PLACE_DIRECT)
        return fail(PT_EINVAL, "direct sums keep no table: not an int32 form (use FP64 or FP32)");
    if (o.init != PT_INIT_RANDOM && o.init != PT_INIT_ORDERED) return fail(PT_EINVAL, "bad init");
    if (o.threads && o.threads != 2 * kMaxSweepThreads &&
        (o.threads % kWave || o.threads < kWave || o.threads > kMaxSweepThreads))
        return fail(PT_EINVAL, "threads must be a multiple of 64 in [64, %d], or %d (overlapped sweep)",
                    kMaxSweepThreads, 2 * kMaxSweepThreads);
    if (o.placement < PT_PLACE_AUTO || o.placement > PT_PLACE_DIRECT) return fail(PT_EINVAL, "bad placement");
    return PT_OK;
}

// Fills the run parameters of c from the options (no device work).
static void ctx_params(pt_ctx *c, int32_t L, int32_t q, double sigma, int32_t R, uint64_t seed, const pt_options &o)
{
    c->L = L; c->q = q; c->R = R; c->prec = o.precision; c->init = o.init; c->sigma = sigma; c->seed = seed;
    c->NT = o.threads ? std::min(o.threads, kMaxSweepThreads) : auto_threads(L);
    c->ser_cap = std::max(0, o.series_capacity);
    c->ev_cap = o.event_capacity > 0 ? o.event_capacity : 4096;
    c->prof = o.profile != 0;
    c->stream = static_cast<hipStream_t>(o.stream);
}

// Device set-up of c in the workspace c->ws (at least the layout's size):
// launch plan, zeroed state, couplings, ladder and bounds, and (draw_spins)
// the initial spins and field table.  Neither allocates nor frees anything.
static pt_status init_core(pt_ctx *c, const double *T, const pt_options &o, bool draw_spins)
{
    const int32_t L = c->L, q = c->q, R = c->R;
    if (hipGetDevice(&c->device) != hipSuccess) return fail(PT_EDEVICE, "no HIP device");
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        return fail(PT_EDEVICE, "device query failed");
    // Field table in LDS when it fits (AUTO, or when asked), else in HBM
    // (AUTO, or when asked); no table when direct sums are asked for.
    const size_t lmax = static_cast<size_t>(lds_max);
    int pl = o.placement == PT_PLACE_DIRECT ? kPlDirect : (o.placement == PT_PLACE_HBM ? kPlHbm : kPlLds);
    bool fits = make_plan(L, q, R, c->prec, false, pl, lmax, c->NT, &c->plan);
    if (!fits && o.placement == PT_PLACE_LDS)
        return fail(PT_EINVAL, "field table of %d x %d entries does not fit in %d B of LDS", q, L, lds_max);
    if (!fits && pl == kPlLds) {
        pl = kPlHbm;
        fits = make_plan(L, q, R, c->prec, false, pl, lmax, c->NT, &c->plan);
    }
    if (!fits) return fail(PT_EINVAL, "couplings and spins of L = %d do not fit in %d B of LDS", L, lds_max);
    bool fused_fits = make_plan(L, q, R, c->prec, true, pl, lmax, c->NT, &c->plan_fused);
    if (!fused_fits && pl == kPlLds && o.placement != PT_PLACE_LDS &&
        make_plan(L, q, R, c->prec, true, kPlHbm, lmax, c->NT, &c->plan_fused)) {
        // keep the persistent launch possible by moving the table to HBM for it
        fused_fits = true;
        pl = kPlHbm;
        make_plan(L, q, R, c->prec, false, pl, lmax, c->NT, &c->plan);
    }
    c->h_in_lds = pl == kPlLds;
    // Overlapped sweep (chain and flush in separate halves of a 512-thread
    // workgroup): FP64 or int32 table in LDS, q <= 4, a whole sweep's draws
    // staged at once, at least four windows per sweep; asked for with threads =
    // 512 (refused where it does not apply).  Not chosen automatically: on the
    // 1024-site, 64-replica workload it ran at 3.10e8 attempts/s against 3.50e8
    // for the plain sweep (same box), its chain slowed by the LDS barriers
    // among its own waves and the extra pass over the previous window's flips.
    const bool ov_ok = pl == kPlLds && c->prec != PT_PREC_F32 && q <= 4 && L >= 256 && L <= 1024;
    if (o.threads == 2 * kMaxSweepThreads && !ov_ok)
        return fail(PT_EINVAL, "the overlapped sweep (threads = %d) needs an FP64 or int32 table in LDS, q <= 4 and "
                    "256 <= L <= 1024", 2 * kMaxSweepThreads);
    if (ov_ok && o.threads == 2 * kMaxSweepThreads) {
        LdsPlan po, pf;
        if (make_plan(L, q, R, c->prec, false, kPlLds, lmax, 2 * kMaxSweepThreads, &po, true) &&
            make_plan(L, q, R, c->prec, true, kPlLds, lmax, 2 * kMaxSweepThreads, &pf, true)) {
            c->plan = po;
            c->plan_fused = pf;
            fused_fits = true;
            c->NT = 2 * kMaxSweepThreads;
        } else {
            return fail(PT_EINVAL, "the overlapped sweep's LDS carve does not fit in %d B", lds_max);
        }
    }

    const Layout lay = layout_of(L, q, R, c->prec, c->ser_cap, c->ev_cap, c->prof);
    if (c->ws_bytes < lay.total) return fail(PT_ENOMEM, "workspace of %zu B < %zu B needed", c->ws_bytes, lay.total);
    Inst &P = c->inst;
    fill_inst(P, c->ws, lay, L, q, R, c->seed,
              o.refresh_every > 0 ? o.refresh_every : 0, c->ser_cap, c->ev_cap, c->prof);
    c->refresh_every = P.refresh_every;

    // zero the (possibly caller-provided) workspace: counters, accumulators
    // and the barrier words start at zero
    pt_status st = zero_async(c->ws, lay.total, c->stream);
    if (st != PT_OK) return st;

    const void *sf = sweep_fn_prec(c->prec, q, c->plan);
    const void *rf = refresh_fn_prec(c->prec, c->plan);
    if ((st = set_lds_attr(sf, c->plan.total)) != PT_OK || (st = set_lds_attr(rf, c->plan.total)) != PT_OK) return st;
    c->can_fuse = false;
    if (fused_fits) {
        const void *sff = sweep_fn_prec(c->prec, q, c->plan_fused);
        int per_cu = 0;
        if (set_lds_attr(sff, c->plan_fused.total) == PT_OK &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sff, c->NT, c->plan_fused.total) == hipSuccess)
            c->can_fuse = static_cast<int64_t>(per_cu) * c->cus >= R;
    }
    c->max_chunk = o.max_sweeps_per_launch > 0 ? o.max_sweeps_per_launch : 1024;

    hipLaunchKernelGGL(k_jstar, dim3((L / 2 + 1 + 255) / 256), dim3(256), 0, c->stream, L, c->sigma,
                       const_cast<double *>(P.J64), const_cast<float *>(P.J32));
    if (hipGetLastError() != hipSuccess) return fail(PT_EDEVICE, "k_jstar launch failed");
    if ((st = setup_instance(c, T)) != PT_OK) return st;
    if (draw_spins) {
        const int64_t total = static_cast<int64_t>(R) * L;
        const int blocks = static_cast<int>(std::min<int64_t>(4096, (total + 255) / 256));
        hipLaunchKernelGGL(k_init_spins, dim3(blocks), dim3(256), 0, c->stream, P,
                           static_cast<int32_t>(c->init == PT_INIT_ORDERED));
        if (hipGetLastError() != hipSuccess) return fail(PT_EDEVICE, "k_init_spins launch failed");
        if ((st = launch_refresh(c)) != PT_OK) return st;
    }
    return PT_OK;
}

static pt_status init_impl(pt_ctx **out, int32_t L, int32_t q, double sigma, const double *T, int32_t R,
                           uint64_t seed, const pt_options *opt, bool draw_spins)
{
    pt_options d;
    pt_default_options(&d);
    const pt_options &o = opt ? *opt : d;
    pt_status st = check_options(o);
    if (st != PT_OK) return st;

    pt_ctx *c = new (std::nothrow) pt_ctx();
    if (!c) return fail(PT_ENOMEM, "host allocation failed");
    ctx_params(c, L, q, sigma, R, seed, o);
    c->T.assign(T, T + R);
    auto bail = [&](pt_status s) {
        if (c->own_ws && c->ws) (void)hipFree(c->ws);
        delete c;
        return s;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(fail(PT_EDEVICE, "no HIP device"));
    const Layout lay = layout_of(L, q, R, c->prec, c->ser_cap, c->ev_cap, c->prof);
    if (o.workspace) {
        if (o.workspace_bytes < lay.total)
            return bail(fail(PT_ENOMEM, "workspace of %zu B < %zu B needed", o.workspace_bytes, lay.total));
        c->ws = static_cast<unsigned char *>(o.workspace);
        c->ws_bytes = o.workspace_bytes;
    } else {
        if (hipMalloc(&c->ws, lay.total) != hipSuccess) return bail(fail(PT_ENOMEM, "hipMalloc(%zu) failed", lay.total));
        c->own_ws = true;
        c->ws_bytes = lay.total;
    }
    if ((st = init_core(c, T, o, draw_spins)) != PT_OK) return bail(st);
    *out = c;
    return PT_OK;
}

pt_status pt_init(pt_ctx **out, int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed,
                  const pt_options *opt)
{
    if (!out) return fail(PT_EINVAL, "out is NULL");
    *out = nullptr;
    const pt_status v = validate(L, q, sigma, T, R);
    if (v != PT_OK) return v;
    return init_impl(out, L, q, sigma, T, R, seed, opt, true);
}

pt_status pt_sweep(pt_ctx *c, int64_t n)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (n < 0) return fail(PT_EINVAL, "n < 0");
    while (n > 0) {
        const int32_t chunk = static_cast<int32_t>(std::min<int64_t>(n, c->max_chunk));
        st = launch_sweep(c, c->sweeps, chunk, 0, 0, c->xsteps, false);
        if (st != PT_OK) return st;
        c->sweeps += chunk;
        c->samples += chunk;
        n -= chunk;
    }
    return PT_OK;
}

pt_status pt_exchange(pt_ctx *c)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    st = launch_exchange(c);
    if (st != PT_OK) return st;
    c->xsteps += 1;
    return PT_OK;
}

pt_status pt_run(pt_ctx *c, int64_t n, int32_t every)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (n < 0 || every < 0) return fail(PT_EINVAL, "n and exchange_every must be >= 0");
    if (every == 0) return pt_sweep(c, n);
    // The schedule counts sweeps from the start of this call: an exchange step
    // follows sweeps every, 2 every, ... of the call, however the sweeps are
    // split into launches.
    if (!c->can_fuse) {
        for (int64_t s = 0; s < n; ++s) {
            if ((st = pt_sweep(c, 1)) != PT_OK) return st;
            if ((s + 1) % every == 0 && (st = pt_exchange(c)) != PT_OK) return st;
        }
        return PT_OK;
    }
    for (int64_t done = 0; done < n;) {
        const int64_t chunk = std::min<int64_t>(n - done, c->max_chunk);
        const int32_t x0 = static_cast<int32_t>(done % every);  // sweeps of the current period already run
        const int64_t nx = (x0 + chunk) / every;                 // exchange steps inside this launch
        st = launch_sweep(c, c->sweeps, static_cast<int32_t>(chunk), every, x0, c->xsteps, true);
        if (st != PT_OK) return st;
        c->sweeps += chunk;
        c->samples += chunk;
        c->xsteps += nx;
        done += chunk;
    }
    return PT_OK;
}

pt_status pt_synchronize(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    HIPCHK(hipStreamSynchronize(c->stream));
    return device_error(c);
}

pt_status pt_observables(pt_ctx *c, pt_obs *o)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!o) return fail(PT_EINVAL, "obs is NULL");
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    HostObs h;
    if ((st = h.fetch(c->inst, c->stream)) != PT_OK) return st;
    h.fill(o, c->sweeps, c->xsteps, c->samples);
    return PT_OK;
}

pt_status pt_get_spins(pt_ctx *c, uint8_t *spins, int32_t *perm)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    const size_t n = static_cast<size_t>(c->R) * c->L;
    if (spins) {
        HIPCHK(hipMemcpy(spins, c->inst.spins, n, hipMemcpyDeviceToHost));
        for (size_t e = 0; e < n; ++e) spins[e] = static_cast<uint8_t>(spins[e] + 1);
    }
    if (perm) HIPCHK(hipMemcpy(perm, c->inst.perm, sizeof(int32_t) * c->R, hipMemcpyDeviceToHost));
    return PT_OK;
}

pt_status pt_get_jstar(pt_ctx *c, double *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!out) return fail(PT_EINVAL, "out is NULL");
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    HIPCHK(hipMemcpy(out, c->inst.J64, sizeof(double) * c->L, hipMemcpyDeviceToHost));
    return PT_OK;
}

pt_status pt_get_series(pt_ctx *c, double *E, double *M, int64_t cap_rows, int64_t *n_out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    const int64_t rows = std::min<int64_t>(std::min<int64_t>(c->sweeps, c->ser_cap), std::max<int64_t>(cap_rows, 0));
    const size_t bytes = sizeof(double) * static_cast<size_t>(rows) * c->R;
    if (E && rows) HIPCHK(hipMemcpy(E, c->inst.serE, bytes, hipMemcpyDeviceToHost));
    if (M && rows) HIPCHK(hipMemcpy(M, c->inst.serM, bytes, hipMemcpyDeviceToHost));
    if (n_out) *n_out = rows;
    return PT_OK;
}

pt_status pt_get_events(pt_ctx *c, pt_event *out, int64_t cap, int64_t *n_out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    unsigned long long n = 0;
    HIPCHK(hipMemcpy(&n, c->inst.ctr + kCtrEvents, sizeof n, hipMemcpyDeviceToHost));
    const int64_t stored = std::min<int64_t>(std::min<int64_t>(static_cast<int64_t>(n), c->ev_cap), std::max<int64_t>(cap, 0));
    if (out && stored) HIPCHK(hipMemcpy(out, c->inst.events, sizeof(pt_event) * stored, hipMemcpyDeviceToHost));
    if (n_out) *n_out = stored;
    return PT_OK;
}

pt_status pt_get_plan(pt_ctx *c, int32_t *placement, int32_t *threads, int32_t *lds_bytes)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    const LdsPlan &p = c->can_fuse ? c->plan_fused : c->plan;
    if (placement) *placement = p.place;
    if (threads) *threads = c->NT;
    if (lds_bytes) *lds_bytes = p.total;
    return PT_OK;
}

pt_status pt_get_phase_counters(pt_ctx *c, uint64_t *out)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!out) return fail(PT_EINVAL, "out is NULL");
    if (!c->prof) return fail(PT_ESTATE, "profiling was not enabled at pt_init (pt_options.profile)");
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    HIPCHK(hipMemcpy(out, c->inst.phase, sizeof(uint64_t) * kPhN * c->R, hipMemcpyDeviceToHost));
    return PT_OK;
}

pt_status pt_reset_stats(pt_ctx *c)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    const Inst &P = c->inst;
    void *arrs[5] = {P.acc6, P.fatt, P.facc, P.xatt, P.xacc};
    const size_t bytes[5] = {sizeof(double) * 6 * c->R, sizeof(int64_t) * c->R, sizeof(int64_t) * c->R,
                             sizeof(int64_t) * c->R, sizeof(int64_t) * c->R};
    for (int a = 0; a < 5; ++a)
        if ((st = zero_async(arrs[a], bytes[a], c->stream)) != PT_OK) return st;
    c->samples = 0;
    return PT_OK;
}

// Checkpoint: header, T, spins (0-based), perm, accumulators.
struct SaveHeader {
    uint32_t magic, version;
    int32_t L, q, R, prec, init, refresh_every;
    uint64_t seed;
    double sigma;
    int64_t sweeps, xsteps, samples;
};

pt_status pt_save(pt_ctx *c, void *buf, size_t *len)
{
    pt_status st = check_ctx(c);
    if (st != PT_OK) return st;
    if (!len) return fail(PT_EINVAL, "len is NULL");
    const int R = c->R, L = c->L;
    const size_t need = sizeof(SaveHeader) + sizeof(double) * R + static_cast<size_t>(R) * L + sizeof(int32_t) * R +
                        sizeof(double) * 6 * R + sizeof(int64_t) * 4 * R;
    if (!buf) {
        *len = need;
        return PT_OK;
    }
    if (*len < need) return fail(PT_EINVAL, "buffer of %zu B < %zu B", *len, need);
    if ((st = pt_synchronize(c)) != PT_OK) return st;
    unsigned char *p = static_cast<unsigned char *>(buf);
    SaveHeader hd{kMagic, kVersion, L, c->q, R, c->prec, c->init, c->refresh_every, c->seed, c->sigma,
                  c->sweeps, c->xsteps, c->samples};
    std::memcpy(p, &hd, sizeof hd); p += sizeof hd;
    std::memcpy(p, c->T.data(), sizeof(double) * R); p += sizeof(double) * R;
    const Inst &P = c->inst;
    HIPCHK(hipMemcpy(p, P.spins, static_cast<size_t>(R) * L, hipMemcpyDeviceToHost)); p += static_cast<size_t>(R) * L;
    HIPCHK(hipMemcpy(p, P.perm, sizeof(int32_t) * R, hipMemcpyDeviceToHost)); p += sizeof(int32_t) * R;
    HIPCHK(hipMemcpy(p, P.acc6, sizeof(double) * 6 * R, hipMemcpyDeviceToHost)); p += sizeof(double) * 6 * R;
    int64_t *arrs[4] = {P.fatt, P.facc, P.xatt, P.xacc};
    for (int a = 0; a < 4; ++a) {
        HIPCHK(hipMemcpy(p, arrs[a], sizeof(int64_t) * R, hipMemcpyDeviceToHost));
        p += sizeof(int64_t) * R;
    }
    *len = need;
    return PT_OK;
}

pt_status pt_load(pt_ctx **out, const void *buf, size_t len, const pt_options *opt)
{
    if (!out || !buf) return fail(PT_EINVAL, "null argument");
    *out = nullptr;
    SaveHeader hd;
    if (len < sizeof hd) return fail(PT_EINVAL, "buffer too short");
    std::memcpy(&hd, buf, sizeof hd);
    if (hd.magic != kMagic || hd.version != kVersion) return fail(PT_EINVAL, "not a checkpoint of this library");
    if (hd.L < 2 || hd.L > 65535 || hd.q < 2 || hd.q > PT_QMAX || hd.R < 1 || hd.R > (1 << 24))
        return fail(PT_EINVAL, "corrupt checkpoint: sizes");
    const int R = hd.R, L = hd.L;
    const size_t need = sizeof hd + sizeof(double) * R + static_cast<size_t>(R) * L + sizeof(int32_t) * R +
                        sizeof(double) * 6 * R + sizeof(int64_t) * 4 * R;
    if (len < need) return fail(PT_EINVAL, "buffer too short");
    const unsigned char *p = static_cast<const unsigned char *>(buf) + sizeof hd;
    std::vector<double> T(R);
    std::memcpy(T.data(), p, sizeof(double) * R); p += sizeof(double) * R;
    pt_status st = validate(L, hd.q, hd.sigma, T.data(), R);
    if (st != PT_OK) return st;
    if (!valid_prec(hd.prec)) return fail(PT_EINVAL, "corrupt checkpoint: precision");
    if (hd.init != PT_INIT_RANDOM && hd.init != PT_INIT_ORDERED) return fail(PT_EINVAL, "corrupt checkpoint: init");
    if (hd.sweeps < 0 || hd.xsteps < 0 || hd.samples < 0) return fail(PT_EINVAL, "corrupt checkpoint: counters");
    // every spin a state 0..q-1 and perm a permutation of 0..R-1, checked on
    // the host before anything reaches the device (kernels index by them)
    {
        const unsigned char *sp = p;
        for (size_t e = 0; e < static_cast<size_t>(R) * L; ++e)
            if (sp[e] >= hd.q)
                return fail(PT_EINVAL, "corrupt checkpoint: spin %zu is %d, not below q = %d", e, sp[e], hd.q);
        int32_t pk = 0;
        std::vector<unsigned char> seen(R, 0);
        for (int k = 0; k < R; ++k) {
            std::memcpy(&pk, sp + static_cast<size_t>(R) * L + sizeof(int32_t) * k, sizeof pk);
            if (pk < 0 || pk >= R || seen[pk]) return fail(PT_EINVAL, "corrupt checkpoint: perm is not a permutation");
            seen[pk] = 1;
        }
    }
    pt_options o;
    if (opt) o = *opt; else pt_default_options(&o);
    o.precision = hd.prec;
    o.init = hd.init;
    if (!opt || !opt->refresh_every) o.refresh_every = hd.refresh_every;
    pt_ctx *c = nullptr;
    if ((st = init_impl(&c, L, hd.q, hd.sigma, T.data(), R, hd.seed, &o, false)) != PT_OK) return st;
    const Inst &P = c->inst;
    std::vector<int32_t> perm(R), slot(R);
    auto fail_free = [&](pt_status s) { pt_free(c); return s; };
    if (hipMemcpy(P.spins, p, static_cast<size_t>(R) * L, hipMemcpyHostToDevice) != hipSuccess)
        return fail_free(fail(PT_EDEVICE, "copy failed"));
    p += static_cast<size_t>(R) * L;
    std::memcpy(perm.data(), p, sizeof(int32_t) * R); p += sizeof(int32_t) * R;
    for (int k = 0; k < R; ++k) slot[perm[k]] = k;  // a permutation (checked above)
    if (hipMemcpy(P.perm, perm.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P.slot_of, slot.data(), sizeof(int32_t) * R, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(P.acc6, p, sizeof(double) * 6 * R, hipMemcpyHostToDevice) != hipSuccess)
        return fail_free(fail(PT_EDEVICE, "copy failed"));
    p += sizeof(double) * 6 * R;
    int64_t *arrs[4] = {P.fatt, P.facc, P.xatt, P.xacc};
    for (int a = 0; a < 4; ++a) {
        if (hipMemcpy(arrs[a], p, sizeof(int64_t) * R, hipMemcpyHostToDevice) != hipSuccess)
            return fail_free(fail(PT_EDEVICE, "copy failed"));
        p += sizeof(int64_t) * R;
    }
    st = launch_refresh(c);
    if (st != PT_OK) return fail_free(st);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail_free(fail(PT_EDEVICE, "refresh failed"));
    c->sweeps = hd.sweeps;
    c->xsteps = hd.xsteps;
    c->samples = hd.samples;
    *out = c;
    return PT_OK;
}

pt_status pt_free(pt_ctx *c)
{
    if (!c) return fail(PT_EINVAL, "null context");
    (void)hipStreamSynchronize(c->stream);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    delete c;
    return PT_OK;
}

// ---------------------------------------------------------------------------
// Single instance without allocation: the device state lives in `scratch`, a
// static device array (one per GPU, held until the process ends).
// ---------------------------------------------------------------------------
}  // extern "C"

static __device__ __align__(256) unsigned char scratch[PT_STATIC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device
// (with that device current).  In host code the array's name only stands in for
// the symbol: kernels and copies must be given this address instead.  The caller
// holds g_scratch_mu[dev].
pt_status scratch_address(int dev, unsigned char **out)
{
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PT_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_run_static(int32_t L, int32_t q, double sigma, const double *T, int32_t R, uint64_t seed, int64_t n,
                        int32_t exchange_every, const pt_options *opt, pt_obs *out, uint8_t *spins_out,
                        int32_t *perm_out)
{
    pt_status st = validate(L, q, sigma, T, R);
    if (st != PT_OK) return st;
    if (n < 0 || exchange_every < 0) return fail(PT_EINVAL, "n and exchange_every must be >= 0");
    pt_options d;
    pt_default_options(&d);
    pt_options o = opt ? *opt : d;
    if (o.workspace) return fail(PT_EINVAL, "pt_run_static takes no workspace (its state lives in the static buffer)");
    if ((st = check_options(o)) != PT_OK) return st;
    o.series_capacity = 0;  // nothing outlives the call but its outputs
    o.profile = 0;
    pt_ctx c;  // on the stack; its temperature copy stays empty (no checkpoints here)
    ctx_params(&c, L, q, sigma, R, seed, o);
    const Layout lay = layout_of(L, q, R, c.prec, c.ser_cap, c.ev_cap, false);
    const size_t need = lay.total + Layout::up(2 * sizeof(double) * static_cast<size_t>(R));
    if (need > PT_STATIC_SCRATCH_BYTES)
        return fail(PT_EINVAL, "state of L = %d, q = %d, R = %d needs %zu B, beyond the static buffer of %zu B", L, q, R,
                    need, static_cast<size_t>(PT_STATIC_SCRATCH_BYTES));
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PT_EDEVICE, "device ordinal %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    unsigned char *base = nullptr;
    if ((st = scratch_address(dev, &base)) != PT_OK) return st;
    c.ws = base;
    c.ws_bytes = lay.total;
    c.own_ws = false;
    if ((st = init_core(&c, T, o, true)) != PT_OK) return st;
    if ((st = pt_run(&c, n, exchange_every)) != PT_OK) return st;
    HIPCHK(hipStreamSynchronize(c.stream));
    if ((st = device_error(&c)) != PT_OK) return st;

    const Inst &P = c.inst;
    hipStream_t s = c.stream;
    if (out) {
        double *Eslot = reinterpret_cast<double *>(base + lay.total);
        double *Mslot = Eslot + R;
        hipLaunchKernelGGL(k_obs_by_slot, dim3((R + 255) / 256), dim3(256), 0, s, P, Eslot, Mslot);
        HIPCHK(hipGetLastError());
        auto get = [&](void *dst, const void *src, size_t bytes) -> pt_status {
            if (dst && bytes) HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s));
            return PT_OK;
        };
        const size_t rd = sizeof(double) * R, ri = sizeof(int64_t) * R, rp = sizeof(int64_t) * (R - 1);
        double *sums[6] = {out->sumE, out->sumE2, out->sumE4, out->sumM, out->sumM2, out->sumM4};
        unsigned long long ctr[kCtrN];
        if ((st = get(out->E, Eslot, rd)) != PT_OK || (st = get(out->M, Mslot, rd)) != PT_OK) return st;
        for (int a = 0; a < 6; ++a)
            if ((st = get(sums[a], P.acc6 + a * R, rd)) != PT_OK) return st;
        if ((st = get(out->flip_att, P.fatt, ri)) != PT_OK || (st = get(out->flip_acc, P.facc, ri)) != PT_OK ||
            (st = get(out->xchg_att, P.xatt, rp)) != PT_OK || (st = get(out->xchg_acc, P.xacc, rp)) != PT_OK ||
            (st = get(out->perm, P.perm, sizeof(int32_t) * R)) != PT_OK || (st = get(ctr, P.ctr, sizeof ctr)) != PT_OK)
            return st;
        HIPCHK(hipStreamSynchronize(s));
        out->R = R; out->q = q; out->L = L;
        out->sweeps = c.sweeps; out->exchange_steps = c.xsteps; out->samples = c.samples;
        out->n_recheck = static_cast<int64_t>(ctr[kCtrRecheck]);
        out->n_banded = static_cast<int64_t>(ctr[kCtrBandedMet] + ctr[kCtrBandedEx]);
        out->n_exact_energy = static_cast<int64_t>(ctr[kCtrExactE]);
        out->n_refresh = static_cast<int64_t>(ctr[kCtrRefresh]);
        out->n_events_dropped = ctr[kCtrEvents] > static_cast<unsigned long long>(c.ev_cap)
                                    ? static_cast<int64_t>(ctr[kCtrEvents] - c.ev_cap)
                                    : 0;
    }
    if (spins_out || perm_out) {
        const size_t ns = static_cast<size_t>(R) * L;
        if (spins_out) HIPCHK(hipMemcpyAsync(spins_out, P.spins, ns, hipMemcpyDeviceToHost, s));
        if (perm_out) HIPCHK(hipMemcpyAsync(perm_out, P.perm, sizeof(int32_t) * R, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (spins_out)
            for (size_t e = 0; e < ns; ++e) spins_out[e] = static_cast<uint8_t>(spins_out[e] + 1);
    }
    return PT_OK;
}

}  // extern "C"

#include "host_jobs.hpp"

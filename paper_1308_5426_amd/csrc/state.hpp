// state.hpp -- device-resident state of one parallel-tempering instance and
// its layout in HBM.  All arrays live in one workspace carved by `Layout`.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace ptmi {

// Global counters (uint64) in Inst::ctr.
enum Counter : int {
    kCtrRecheck = 0,     // FP64 direct rechecks of near-threshold attempts
    kCtrBandedMet = 1,   // Metropolis decisions inside the band
    kCtrBandedEx = 2,    // exchange decisions inside the band
    kCtrExactE = 3,      // exact energies computed for uncertain exchanges
    kCtrRefresh = 4,     // field recomputations
    kCtrEvents = 5,      // events logged (may exceed capacity)
    kCtrError = 6,       // error bits (kErr*)
    kCtrBarCount = 8,    // grid barrier arrivals (uint32 in the low word)
    kCtrBarGen = 9,      // grid barrier generation
    kCtrN = 16
};
enum : unsigned long long { kErrBarrierTimeout = 1ull, kErrBadLaunch = 2ull };

// Per-walker phase counters (uint64, Inst::phase[w * kPhN + k]), kept when
// profiling is on: shader-clock cycles spent by the walker's workgroup in each
// phase of its sweeps (read by thread 0 right after the barrier that closes
// the phase), and event counts.
enum Phase : int {
    kPhDraw = 0,        // generating the chunk's draws
    kPhChain = 1,       // the Metropolis chain through the windows
    kPhFlush = 2,       // applying the windows' flips to the field table
    kPhRecord = 3,      // end-of-sweep sums, observables and scheduled refreshes
    kPhExchange = 4,    // arrival at the device barrier to leaving it (exchange included)
    kPhTotal = 5,       // the whole walker loop of the launch
    kPhWindows = 6,     // windows of 64 attempts
    kPhFlushes = 7,     // windows with at least one flip to apply
    kPhFlips = 8,       // accepted flips
    kPhIters = 9,       // guess-and-check iterations of the chain
    // the chain's cycles by step of its iterations (part of kPhChain):
    kPhCGuess = 10,     // the guess: sure accepts, same-site cut, compaction
    kPhCCorr = 11,      // the guessed flips applied to later lanes' dE
    kPhCCheck = 12,     // re-decisions, commits and counters
    kPhCResolve = 13,   // the first differing lane decided, later lanes rebuilt
    kPhCRedo = 14,      // lanes whose site an earlier flip changed, dE re-derived
    kPhCSync = 15,      // the workgroup barrier closing an iteration
    kPhN = 16
};

// Table precisions (values of PT_PREC_*).
enum : int { kPrecF64 = 0, kPrecF32 = 1, kPrecI32 = 2 };

// Rigorous error bounds of a field table (see sweep.hpp), in table units
// (the real value of a table entry is entry * qscale).  Per entry: right after
// a refresh the table holds the sum of at most L couplings in its precision,
// off the exact field by at most init; each flip applied since then adds one
// rounded coupling and one rounding of the sum (unit).  nupd_max caps the
// number of flips between refreshes so the drift stays below 1e-3 S.  The
// walker's tracked energy is off the exact one by at most ebound (real units)
// right after a refresh, plus flipE per accepted flip; FP64 tables instead add
// the chain's own bound of each accepted energy change.
//   FP64: FP64 couplings summed in FP64.
//   FP32: FP32 couplings J32 summed in FP64 (so the table holds the FP32
//         couplings' fields, off the exact ones by at most D32 = sum_r |J*(r) -
//         J32(r)| plus rounding), and energies from sums of J32: the energy of
//         the J32 couplings, off the exact one by at most L D32 / 2.
//   I32:  couplings quantised to integers Jq(r) = rint(J*(r) 2^k), k the
//         largest with S 2^k + L < 2^31 - 2 (so no field overflows), qscale =
//         2^-k; integer sums and updates are exact, so the table holds the
//         quantised couplings' fields exactly: off the exact fields by at most
//         Dq = sum_r |J*(r) - Jq(r) 2^-k|, with no drift and no refresh; the
//         energy, tracked exactly in the quantised couplings, is off by at
//         most L Dq / 2.
// S = sum_r J*(r), Jmax = J*(1).
//
// The table keeps rows 0 .. q-2 only: a site's q fields sum to the coupling
// sum of the table's own couplings, Stab (FP64 or FP32 couplings summed in
// FP64, or the quantised ones, exactly), so row q-1 is Stab minus the others.
// An energy change read from the table is a difference of two entries; when
// one of them is the implicit row its error is at most that of q - 1 entries,
// plus Stab's own error and q roundings of the subtraction (none for int
// tables, whose sums are exact and whose implicit entry deviates from the
// exact field by at most Dq like any other).  So the chain's starting bound is
// rows (init + nupd unit) + impl with rows = q + 1 and impl = (L + q + 2) 2^-53
// S (FP tables; rows = 2, impl = 0 for int32).
struct TableBounds {
    double init, unit;
    int64_t nupd_max;
    double flipE, ebound, qscale;
    double hsum;        // Stab in table units
    double rows, impl;  // the chain's starting bound: rows (init + nupd unit) + impl
};

__host__ __device__ inline TableBounds table_bounds(double S, double Jmax, double D32, double Dq, int L, int prec,
                                                    double qscale, int q, double Stab)
{
    const double u64 = 0x1p-53, Ld = static_cast<double>(L);
    TableBounds b;
    b.qscale = 1.0;
    b.flipE = 0.0;
    b.ebound = 0.0;
    b.hsum = Stab;
    b.rows = prec == kPrecI32 ? 2.0 : static_cast<double>(q + 1);
    b.impl = prec == kPrecI32 ? 0.0 : (Ld + static_cast<double>(q) + 2.0) * u64 * S * 1.01;
    if (prec == kPrecI32) {
        b.qscale = qscale;
        b.init = Dq / qscale * 1.01;  // table units
        b.unit = 0.0;
        b.nupd_max = static_cast<int64_t>(4e18);
        b.ebound = 0.5 * Ld * Dq * 1.01 + Ld * Ld * u64 * S;
        return b;
    }
    const double uF = prec == kPrecF32 ? 0x1p-24 : u64;
    const double Dc = prec == kPrecF32 ? D32 : 0.0;
    b.init = (uF * S + Dc + (Ld + 4.0) * u64 * S) * 1.01 + 1e-15 * S;
    b.unit = uF * (1.001 * S + 2.0 * Jmax) * 1.01 + u64 * S;
    const double cap = 1e-3 * S / b.unit;
    b.nupd_max = cap > 4.0e18 ? static_cast<int64_t>(4e18) : static_cast<int64_t>(cap);
    if (prec == kPrecF32) {
        b.flipE = (Ld + 512.0) * u64 * 1.001 * S * 1.01;
        b.ebound = (0.5 * Ld * D32 + Ld * Ld * u64 * S) * 1.01;
    }
    return b;
}

struct Event {
    int64_t a, b, c;
    int32_t kind, decision;
    double x;
};

// One instance (job): R walkers on a ring of L sites with q states.
// Walker-indexed arrays: spins, h, E, Eerr, nupd, counts, Mw.
// Slot-indexed arrays: beta, perm, acc6, fatt, facc; pair-indexed: xatt, xacc.
struct Inst {
    int32_t L, q, R, walker0;  // walker0: global id offset of walker 0 (batched jobs)
    uint32_t key0, key1;
    int32_t refresh_every;     // 0 = never on schedule
    int32_t ser_cap;           // series rows kept
    int64_t nupd_max;          // forced refresh when the drift counter exceeds this
    double bound_init;         // bound on |h_table - h_exact| right after a refresh
    double bound_unit;         // added to that bound by each applied flip
    double bound_flipE;        // energy error per accepted flip of an FP32 table (0 otherwise)
    double ebound;             // energy error right after a refresh (0: FP64 table)
    double qscale;             // real value of one table unit (2^-k for I32, else 1)
    double hsum;               // sum of a site's q fields (table units): row q-1 = hsum - rows 0..q-2
    double bound_rows, bound_impl;  // the chain's starting bound: rows (init + nupd unit) + impl
    const double *J64;         // [L]
    const float *J32;          // [L]
    const int32_t *Jq;         // [L] quantised couplings (I32 tables)
    uint8_t *spins;            // [R][L], states 0..q-1
    void *h;                   // [R][q-1][L] field table backing store (double, float or int32)
    double *E, *Eerr;          // [R] tracked energy and a rigorous bound on its error
    int64_t *nupd;             // [R] flips applied to the table since its last refresh
    int32_t *counts;           // [R][kQMax] number of sites per state
    double *Mw;                // [R] magnetisation
    int32_t *perm, *slot_of;   // [R] slot -> walker, walker -> slot
    const double *beta;        // [R] by slot
    double *acc6;              // [6][R] sums of E, E^2, E^4, M, M^2, M^4 by slot
    int64_t *fatt, *facc;      // [R] by slot
    int64_t *xatt, *xacc;      // [R] by pair
    double *serE, *serM;       // [ser_cap][R] by slot
    Event *events;
    int32_t ev_cap;
    unsigned long long *ctr;   // [kCtrN]
    TableBounds *bnd;          // bounds computed on the device (job kernel)
    unsigned long long *phase; // [R][kPhN] phase counters, or null (profiling off)
};

struct Layout {
    size_t J64, J32, Jq, spins, h, E, Eerr, nupd, counts, Mw, perm, slot_of, beta, acc6, fatt, facc,
        xatt, xacc, serE, serM, events, ctr, bnd, T, phase, total;

    static size_t up(size_t x) { return (x + 255) & ~static_cast<size_t>(255); }

    Layout(int L, int q, int R, size_t fbytes, int ser_cap, int ev_cap, bool prof = false)
    {
        size_t o = 0;
        auto take = [&](size_t bytes) {
            const size_t at = o;
            o += up(bytes);
            return at;
        };
        J64 = take(sizeof(double) * L);
        J32 = take(sizeof(float) * L);
        Jq = take(sizeof(int32_t) * L);
        spins = take(static_cast<size_t>(R) * L);
        h = take(fbytes * static_cast<size_t>(R) * (q - 1) * L);  // row q-1 is implicit
        E = take(sizeof(double) * R);
        Eerr = take(sizeof(double) * R);
        nupd = take(sizeof(int64_t) * R);
        counts = take(sizeof(int32_t) * R * 16);
        Mw = take(sizeof(double) * R);
        perm = take(sizeof(int32_t) * R);
        slot_of = take(sizeof(int32_t) * R);
        beta = take(sizeof(double) * R);
        acc6 = take(sizeof(double) * 6 * R);
        fatt = take(sizeof(int64_t) * R);
        facc = take(sizeof(int64_t) * R);
        xatt = take(sizeof(int64_t) * R);
        xacc = take(sizeof(int64_t) * R);
        serE = take(sizeof(double) * static_cast<size_t>(ser_cap) * R);
        serM = take(sizeof(double) * static_cast<size_t>(ser_cap) * R);
        events = take(sizeof(Event) * static_cast<size_t>(ev_cap));
        ctr = take(sizeof(unsigned long long) * kCtrN);
        bnd = take(sizeof(TableBounds));
        T = take(sizeof(double) * R);
        phase = take(prof ? sizeof(unsigned long long) * kPhN * static_cast<size_t>(R) : 0);
        total = o;
    }
};

}  // namespace ptmi

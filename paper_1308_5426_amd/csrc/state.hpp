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
    kPhN = 10
};

// Rigorous error bounds of a field table (see sweep.hpp).  Per entry: right
// after a refresh the FP64 sum of at most L couplings is rounded to the
// table's precision (init); each flip applied since then adds one rounded
// coupling and one rounding of the sum (unit).  S = sum_r J*(r), Jmax = J*(1).
// nupd_max caps the number of flips between refreshes so the drift stays below
// 1e-3 S.  FP32 tables take a walker's energy change from the flush's FP64 sums
// of the FP32 couplings, sum_j J32(|i-j|)([s_j=a] - [s_j=b]): per accepted flip
// that is off by at most D32 = sum_r |J*(r) - J32(r)| plus the FP64 rounding of
// an L-term sum (flipE; 0 for FP64 tables, whose energy changes carry their
// own bound).
struct TableBounds {
    double init, unit;
    int64_t nupd_max;
    double flipE;
};

__host__ __device__ inline TableBounds table_bounds(double S, double Jmax, double D32, int L, bool f32)
{
    const double u64 = 0x1p-53;
    const double uF = f32 ? 0x1p-24 : u64;
    TableBounds b;
    b.init = (uF * S + (static_cast<double>(L) + 4.0) * u64 * S) * 1.01 + 1e-15 * S;
    b.unit = uF * (1.001 * S + 2.0 * Jmax) * 1.01 + u64 * S;
    const double cap = 1e-3 * S / b.unit;
    b.nupd_max = cap > 4.0e18 ? static_cast<int64_t>(4e18) : static_cast<int64_t>(cap);
    b.flipE = f32 ? (D32 + (static_cast<double>(L) + 512.0) * u64 * 1.001 * S) * 1.01 : 0.0;
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
    const double *J64;         // [L]
    const float *J32;          // [L]
    uint8_t *spins;            // [R][L], states 0..q-1
    void *h;                   // [R][q][L] field table backing store (float or double)
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
    size_t J64, J32, spins, h, E, Eerr, nupd, counts, Mw, perm, slot_of, beta, acc6, fatt, facc,
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
        spins = take(static_cast<size_t>(R) * L);
        h = take(fbytes * static_cast<size_t>(R) * q * L);
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

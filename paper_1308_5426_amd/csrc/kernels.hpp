// kernels.hpp -- host-side handles of the gfx950 kernels by table
// precision.  Each precision's kernel variants (sweep, refresh, batch/serve)
// are instantiated in a source file of their own (kernels_f64.hip,
// kernels_f32.hip, kernels_i32.hip), so the variants build in parallel; the
// functions below return the launchable kernel for a plan.
#pragma once
#include "jobs.hpp"

namespace ptmi {

const void *sweep_kernel_f64(int q, const LdsPlan &p);
const void *sweep_kernel_f32(int q, const LdsPlan &p);
const void *sweep_kernel_i32(int q, const LdsPlan &p);
const void *refresh_kernel_f64(const LdsPlan &p);
const void *refresh_kernel_f32(const LdsPlan &p);
const void *refresh_kernel_i32(const LdsPlan &p);
const void *jobs_kernel_f64();
const void *jobs_kernel_f32();
const void *jobs_kernel_i32();

#ifdef PTMI_KERNEL_SELECT
// Kernel variant by the number of states (two, four, six or eight flush rows
// in registers for the q - 1 stored rows of q <= 3, 4, 6 or 8; row by row
// beyond), by where the field table lives and by whether the FP64 couplings
// are in LDS.  The two- and four-row forms read their coefficients from a
// table that covers states below 4.
template <typename F, int PL, bool J64L>
const void *sweep_fn_q(int q)
{
    if constexpr (PL == kPlDirect) return reinterpret_cast<const void *>(&k_sweep<F, 0, PL, J64L>);
    if (q <= 3) return reinterpret_cast<const void *>(&k_sweep<F, 2, PL, J64L>);
    if (q <= 4) return reinterpret_cast<const void *>(&k_sweep<F, 4, PL, J64L>);
    if (q <= 6) return reinterpret_cast<const void *>(&k_sweep<F, 6, PL, J64L>);
    if (q <= 8) return reinterpret_cast<const void *>(&k_sweep<F, 8, PL, J64L>);
    return reinterpret_cast<const void *>(&k_sweep<F, 0, PL, J64L>);
}
template <typename F, int PL>
const void *sweep_fn_j(int q, const LdsPlan &p)
{
    if constexpr (table_prec<F>() == kPrecF64)  // FP64 couplings are the table's own, always in LDS
        return sweep_fn_q<F, PL, true>(q);
    else if constexpr (table_prec<F>() == kPrecI32)  // never in LDS
        return sweep_fn_q<F, PL, false>(q);
    else
        return p.j64_in_lds ? sweep_fn_q<F, PL, true>(q) : sweep_fn_q<F, PL, false>(q);
}
template <typename F>
const void *sweep_fn(int q, const LdsPlan &p)
{
    if constexpr (table_prec<F>() != kPrecF32) {  // overlapped sweep: FP64 / int32 table in LDS, q <= 4
        if (p.ovl) {
            if constexpr (table_prec<F>() == kPrecF64)
                return reinterpret_cast<const void *>(&k_sweep<F, 4, kPlLds, true, true>);
            else
                return reinterpret_cast<const void *>(&k_sweep<F, 4, kPlLds, false, true>);
        }
    }
    switch (p.place) {
    case kPlLds: return sweep_fn_j<F, kPlLds>(q, p);
    case kPlHbm: return sweep_fn_j<F, kPlHbm>(q, p);
    default:
        if constexpr (table_prec<F>() == kPrecI32) return nullptr;  // no table: not an int form
        else return sweep_fn_j<F, kPlDirect>(q, p);
    }
}
template <typename F, int PL>
const void *refresh_fn_j(const LdsPlan &p)
{
    if constexpr (table_prec<F>() == kPrecF64) return reinterpret_cast<const void *>(&k_refresh<F, PL, true>);
    else if constexpr (table_prec<F>() == kPrecI32) return reinterpret_cast<const void *>(&k_refresh<F, PL, false>);
    else
        return p.j64_in_lds ? reinterpret_cast<const void *>(&k_refresh<F, PL, true>)
                            : reinterpret_cast<const void *>(&k_refresh<F, PL, false>);
}
template <typename F>
const void *refresh_fn(const LdsPlan &p)
{
    // refreshes of an HBM table and of a direct-sum walker (whose HBM table is
    // never read) run the same code
    return p.place == kPlLds ? refresh_fn_j<F, kPlLds>(p) : refresh_fn_j<F, kPlHbm>(p);
}
#endif  // PTMI_KERNEL_SELECT

}  // namespace ptmi

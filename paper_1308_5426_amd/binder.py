"""Critical temperature of the q = 3 ring from Binder-cumulant crossings.

Paper, section 5.1: each ring size L is simulated by parallel tempering over a
uniform temperature grid; after thermalization the production sweeps give
V_M(T) = 1 - <M^4> / (3 <M^2>^2) (eq. 12) per temperature, and the crossing of
the curves of two sizes estimates T_c, listed per sigma in Table 1.  Here the
production run is cut into blocks (moment sums read and cleared after each),
and the error of V_M comes from the jackknife over the blocks.

    python -m paper_1308_5426_amd.binder --sigma 0.6 --sizes 512,1024,2048

prints one JSON line: the crossings of every pair of sizes, their mean, and the
value Table 1 gives for that sigma.  With --energy-cumulant it also takes the
maximum over temperature of U_E = <E^4>/<E^2>^2 (eq. 11) per size and fits
U_E,max(L) = U_E(inf) + A L^-B by Levenberg-Marquardt, to compare with Table 2.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import Simulation
from .analysis import binder_crossings, binder_cumulant, energy_cumulant, jackknife, power_law_fit

# Table 2: extrapolated fourth-order energy cumulant (q = 3)
TABLE2_UE = {0.5: 1.022, 0.6: 1.0066, 0.65: 1.0021, 0.7: 1.0007, 0.72: 1.0006, 0.74: 1.0002, 0.76: 0.9999,
             0.78: 0.9999}

# Table 1: critical temperatures in the thermodynamic limit (q = 3)
TABLE1_TC = {0.2: 3.955, 0.3: 2.7175, 0.4: 2.085, 0.5: 1.6875, 0.6: 1.4125, 0.7: 1.20, 0.8: 1.03}


def binder_curve(L, sigma, T, therm, prod, blocks, seed, q=3, log=None, with_energy=False):
    """V_M per temperature (ascending T) with jackknife errors over `blocks`
    production blocks, and the exchange acceptance per neighbour pair; with
    with_energy, also U_E = <E^4>/<E^2>^2 (eq. 11) and its errors."""
    t0 = time.time()
    sim = Simulation(L, q, sigma, T, seed)
    try:
        sim.run(therm, 1)
        sim.reset_stats()
        per = max(1, prod // blocks)
        M2, M4, E2, E4, xatt, xacc = [], [], [], [], 0, 0
        for b in range(blocks):
            sim.run(per, 1)
            o = sim.observables()
            sim.reset_stats()
            n = float(o["samples"])
            M2.append(o["sumM2"] / n)
            M4.append(o["sumM4"] / n)
            E2.append(o["sumE2"] / n)
            E4.append(o["sumE4"] / n)
            xatt = xatt + o["xchg_att"]
            xacc = xacc + o["xchg_acc"]
            if log:
                log(f"L={L}: block {b + 1}/{blocks} done, {time.time() - t0:.1f} s")
    finally:
        sim.close()
    V, dV = jackknife({"M2": np.array(M2), "M4": np.array(M4)},
                      lambda m: binder_cumulant(m["M2"], m["M4"]), nbins=blocks)
    xr = np.asarray(xacc) / np.maximum(np.asarray(xatt), 1)
    if with_energy:
        U, dU = jackknife({"E2": np.array(E2), "E4": np.array(E4)},
                          lambda m: energy_cumulant(m["E2"], m["E4"]), nbins=blocks)
        return np.asarray(V), np.asarray(dV), xr, time.time() - t0, np.asarray(U), np.asarray(dU)
    return np.asarray(V), np.asarray(dV), xr, time.time() - t0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sigma", type=float, default=0.6)
    ap.add_argument("--sizes", default="512,1024,2048")
    ap.add_argument("--tmin", type=float, default=1.30)
    ap.add_argument("--tmax", type=float, default=1.55)
    ap.add_argument("--replicas", type=int, default=64)
    ap.add_argument("--therm", type=int, default=20000)
    ap.add_argument("--prod", type=int, default=50000)
    ap.add_argument("--blocks", type=int, default=20)
    ap.add_argument("--seed", type=int, default=1234)
    ap.add_argument("--energy-cumulant", action="store_true",
                    help="also the maximum of U_E per size and its extrapolation U + A L^-B (Table 2)")
    a = ap.parse_args(argv)
    sizes = [int(s) for s in a.sizes.split(",")]
    T = np.linspace(a.tmin, a.tmax, a.replicas)

    def log(msg):
        print(msg, file=sys.stderr, flush=True)

    curves, out, umax = {}, {}, {}
    for L in sizes:
        r = binder_curve(L, a.sigma, T, a.therm, a.prod, a.blocks, a.seed, log=log, with_energy=a.energy_cumulant)
        V, dV, xr, dt = r[:4]
        curves[L] = (T, V)
        out[str(L)] = {"V_M": [round(float(v), 5) for v in V], "dV_M": [round(float(v), 5) for v in dV],
                       "min_exchange_acceptance": round(float(np.min(xr)), 4), "seconds": round(dt, 1)}
        if a.energy_cumulant:
            U, dU = r[4], r[5]
            k = int(np.argmax(U))
            umax[L] = (float(U[k]), float(dU[k]), float(T[k]))
            out[str(L)]["U_E_max"] = [round(umax[L][0], 6), round(umax[L][1], 6), round(umax[L][2], 5)]
    est, pairs = binder_crossings(curves)
    res = {"sigma": a.sigma, "q": 3, "sizes": sizes, "T": [round(float(t), 5) for t in T],
           "therm": a.therm, "prod": a.prod, "blocks": a.blocks,
           "crossings": {f"{p[0]}-{p[1]}": round(t, 4) for p, t in pairs.items()},
           "Tc_estimate": None if est is None else round(est, 4),
           "Tc_table1": TABLE1_TC.get(round(a.sigma, 2)), "curves": out}
    if a.energy_cumulant and len(sizes) >= 3:
        Ls = sorted(umax)
        try:
            popt, perr = power_law_fit(Ls, [umax[L][0] for L in Ls], sigma=[max(umax[L][1], 1e-9) for L in Ls])
            res["U_E_inf"] = [round(float(popt[0]), 6), round(float(perr[0]), 6)]
            res["U_E_fit_A_B"] = [float(popt[1]), float(popt[2])]
        except Exception as e:  # a fit that does not converge is reported, not hidden
            res["U_E_inf"] = f"fit failed: {e}"
        res["U_E_inf_table2"] = TABLE2_UE.get(round(a.sigma, 2))
    print(json.dumps(res))


if __name__ == "__main__":
    main()

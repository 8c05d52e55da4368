"""Thermodynamic analysis of parallel-tempering output (host side).

Paper, section 5.1: the fourth-order energy cumulant U_E = <E^4>/<E^2>^2
(eq. 11), the Binder cumulant V_M = 1 - <M^4>/(3 <M^2>^2) (eq. 12), error bars
by the jackknife, the critical temperature from the crossing of V_M(T) curves
of different ring sizes, and the extrapolation U_E,max(L) = U_inf + A L^-B
fitted by Levenberg-Marquardt.  Inputs are the per-slot moment sums or the
per-sweep series that the GPU library records; nothing here touches the GPU.
"""
from __future__ import annotations

import numpy as np


def energy_cumulant(E2, E4):
    """U_E = <E^4> / <E^2>^2 (eq. 11) from the two means."""
    return np.asarray(E4) / np.asarray(E2) ** 2


def binder_cumulant(M2, M4):
    """V_M = 1 - <M^4> / (3 <M^2>^2) (eq. 12) from the two means."""
    return 1.0 - np.asarray(M4) / (3.0 * np.asarray(M2) ** 2)


def from_sums(obs):
    """Per-slot means and cumulants from the library's moment sums."""
    n = float(obs["samples"])
    m = {k: np.asarray(obs["sum" + k]) / n for k in ("E", "E2", "E4", "M", "M2", "M4")}
    m["U_E"] = energy_cumulant(m["E2"], m["E4"])
    m["V_M"] = binder_cumulant(m["M2"], m["M4"])
    return m


def jackknife(series, stat, nbins=32):
    """Jackknife mean and error of stat(block means) over nbins contiguous bins
    of the leading axis of `series` (e.g. sweeps).  stat maps a dict of block
    means to a value; series is a dict name -> array [n, ...]."""
    n = len(next(iter(series.values())))
    nbins = max(2, min(nbins, n))
    edges = np.linspace(0, n, nbins + 1).astype(int)
    bins = {k: np.stack([v[edges[b]:edges[b + 1]].mean(axis=0) for b in range(nbins)]) for k, v in series.items()}
    full = stat({k: v.mean(axis=0) for k, v in bins.items()})
    leave = np.stack([stat({k: (v.sum(axis=0) - v[b]) / (nbins - 1) for k, v in bins.items()})
                      for b in range(nbins)])
    mean = nbins * np.asarray(full) - (nbins - 1) * leave.mean(axis=0)
    err = np.sqrt((nbins - 1) / nbins * ((leave - leave.mean(axis=0)) ** 2).sum(axis=0))
    return mean, err


def cumulants_with_errors(E, M, nbins=32):
    """U_E and V_M per slot with jackknife errors from per-sweep series [n][R]."""
    s = {"E2": np.asarray(E) ** 2, "E4": np.asarray(E) ** 4, "M2": np.asarray(M) ** 2, "M4": np.asarray(M) ** 4}
    ue = jackknife(s, lambda b: energy_cumulant(b["E2"], b["E4"]), nbins)
    vm = jackknife(s, lambda b: binder_cumulant(b["M2"], b["M4"]), nbins)
    return ue, vm


def crossing(T1, V1, T2, V2):
    """Temperature where two curves V(T) (sampled on ascending grids) cross,
    by linear interpolation of their difference on the union grid.  Returns
    the first crossing, or None."""
    T = np.union1d(np.asarray(T1, float), np.asarray(T2, float))
    lo, hi = max(np.min(T1), np.min(T2)), min(np.max(T1), np.max(T2))
    T = T[(T >= lo) & (T <= hi)]
    d = np.interp(T, T1, V1) - np.interp(T, T2, V2)
    for k in range(len(T) - 1):
        if d[k] == 0.0:
            return float(T[k])
        if d[k] * d[k + 1] < 0.0:
            return float(T[k] - d[k] * (T[k + 1] - T[k]) / (d[k + 1] - d[k]))
    return None


def binder_crossings(curves):
    """curves: {L: (T, V_M)}.  Crossings of every pair of sizes, and their
    mean as the estimate of T_c (paper, section 5.1)."""
    Ls = sorted(curves)
    out = {}
    for a in range(len(Ls)):
        for b in range(a + 1, len(Ls)):
            t = crossing(*curves[Ls[a]], *curves[Ls[b]])
            if t is not None:
                out[(Ls[a], Ls[b])] = t
    est = float(np.mean(list(out.values()))) if out else None
    return est, out


def power_law_fit(L, U, sigma=None, p0=None):
    """Fit U(L) = U_inf + A L^-B by Levenberg-Marquardt (scipy's curve_fit,
    method 'lm'); returns (U_inf, A, B) and their standard errors."""
    from scipy.optimize import curve_fit

    L = np.asarray(L, float)
    U = np.asarray(U, float)

    def f(x, u, a, b):
        return u + a * x ** (-b)

    if p0 is None:
        p0 = (U[-1], (U[0] - U[-1]) * L[0], 1.0)
    popt, pcov = curve_fit(f, L, U, p0=p0, sigma=sigma, absolute_sigma=sigma is not None, method="lm",
                           maxfev=20000)
    return popt, np.sqrt(np.diag(pcov))

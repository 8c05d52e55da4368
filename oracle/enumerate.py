"""Exact Boltzmann averages of small long-range Potts rings by full enumeration.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For L <= 8 and q <= 3 every one of the q^L states is listed; the energy of each
is eq. 2 with each unordered pair once, the magnetisation is eq. 10.  Parallel
tempering's stationary law is the product of the Boltzmann laws of the slots,
so the acceptance rate of an exchange attempt between slots k and k+1
(eq. 9) is the double sum over the two energy distributions of
min(1, exp((E - E')(beta_k - beta_{k+1}))).
"""
from __future__ import annotations

import itertools

import numpy as np


def states(L: int, q: int) -> np.ndarray:
    """All q^L spin configurations, values 1..q, shape (q^L, L)."""
    return np.array(list(itertools.product(range(1, q + 1), repeat=L)), dtype=np.int64)


def energies(J: np.ndarray, S: np.ndarray) -> np.ndarray:
    """E(s) = -sum_{i<j} J*(j-i) delta(s_i, s_j) for every row of S."""
    L = S.shape[1]
    E = np.zeros(S.shape[0])
    for i in range(L):
        for j in range(i + 1, L):
            E -= J[j - i] * (S[:, i] == S[:, j])
    return E


def magnetisations(q: int, S: np.ndarray) -> np.ndarray:
    L = S.shape[1]
    counts = np.stack([(S == k).sum(axis=1) for k in range(1, q + 1)], axis=1)
    return (q * counts.max(axis=1) / L - 1.0) / (q - 1.0)


def boltzmann_moments(J, q, betas):
    """Exact <E>, <E^2>, <E^4>, <M>, <M^2>, <M^4> per inverse temperature."""
    S = states(len(J), q)
    E = energies(np.asarray(J), S)
    M = magnetisations(q, S)
    out = []
    for b in betas:
        w = np.exp(-b * (E - E.min()))
        w /= w.sum()
        out.append(dict(E=w @ E, E2=w @ E**2, E4=w @ E**4, M=w @ M, M2=w @ M**2, M4=w @ M**4))
    return out, E


def exchange_rates(J, q, betas):
    """Exact acceptance probability of an exchange attempt between neighbouring slots."""
    S = states(len(J), q)
    E = energies(np.asarray(J), S)
    levels, mult = np.unique(np.round(E, 12), return_counts=True)
    rates = []
    for k in range(len(betas) - 1):
        b0, b1 = betas[k], betas[k + 1]
        p0 = mult * np.exp(-b0 * (levels - levels.min())); p0 /= p0.sum()
        p1 = mult * np.exp(-b1 * (levels - levels.min())); p1 /= p1.sum()
        d = (levels[:, None] - levels[None, :]) * (b0 - b1)
        rates.append(float(p0 @ np.minimum(1.0, np.exp(np.minimum(d, 0.0))) @ p1))
    return np.array(rates)

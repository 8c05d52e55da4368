"""Inputs that put one decision inside the 1e-9 band, built from the oracle.

TEST INFRASTRUCTURE (imported by the tests only).  Each case picks a seed and
sets a temperature so that a chosen decision sits exactly at its threshold:

* Metropolis (eq. 8): attempt 0 of sweep 0 of walker 0 proposes i: a -> b
  with energy change dE > 0 and uniform u; slot 0 gets T_0 = dE / (-ln u),
  so beta_0 dE + ln u = 0 up to rounding.
* Exchange (eq. 9): right after initialisation walkers 0 and 1 have energies
  E_0 < E_1; the first exchange attempt (step 0, stage 0, pair (0, 1)) draws
  u; beta_1 = beta_0 - ln u / (E_0 - E_1) makes ln u - (E_0 - E_1)(beta_0 -
  beta_1) = 0 up to rounding.

The draws come from the oracle's Philox (pinned by known-answer vectors) and
dE from two full energies (pinned by closed forms and brute force), not from
the sweep code under test.
"""
from __future__ import annotations

import math

import numpy as np


def _draws(orc, seed, ctr):
    key = [seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF]
    return [int(x) for x in orc.philox4x32_10(ctr, key)]


def _unit(hi, lo):
    return (((hi << 20) | (lo >> 12)) + 0.5) * 2.0**-52


def metropolis_case(orc, L=24, q=3, sigma=0.5, R=4, seed0=1):
    """(seed, T ladder, (i, a, b, dE, u)) with attempt (w=0, n=0, t=0) at its threshold."""
    J = orc.jstar(L, sigma)
    for seed in range(seed0, seed0 + 1000):
        s0 = orc.PT(L, q, sigma, [1.0], seed).spins()[0].astype(np.int64)
        o = _draws(orc, seed, [0, 0, 0, 0])
        i = (o[0] * L) >> 32
        k = 1 + ((o[1] * (q - 1)) >> 32)
        u = _unit(o[2], o[3])
        a = int(s0[i])
        b = (a - 1 + k) % q + 1
        s1 = s0.copy()
        s1[i] = b
        dE = orc.energy(J, s1) - orc.energy(J, s0)
        if dE > 1e-2 and -math.log(u) > 1e-2:
            T0 = dE / -math.log(u)
            T = np.array([T0 * 1.6**r for r in range(R)])
            return seed, T, (int(i), a, b, dE, u)
    raise RuntimeError("no seed found")


def exchange_case(orc, L=24, q=3, sigma=0.5, seed0=1):
    """(seed, T ladder [T_0, T_1]) with the first exchange attempt at its threshold."""
    for seed in range(seed0, seed0 + 1000):
        E = orc.PT(L, q, sigma, [1.0, 2.0], seed).energies()
        o = _draws(orc, seed, [0, 0, 0, 1])
        lnu = math.log(_unit(o[0], o[1]))
        d = E[0] - E[1]
        if d < 0 and -lnu < 0.8 * -d:
            beta1 = 1.0 - lnu / d
            return seed, np.array([1.0, 1.0 / beta1])
    raise RuntimeError("no seed found")

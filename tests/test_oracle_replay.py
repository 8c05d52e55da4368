"""Pins of the oracle's banded-replay protocol and of its moment accumulators.

* A decision placed exactly at its threshold (see banded_cases) must be
  counted as banded; replaying decision 0 or 1 for its key must give the two
  different trajectories, one of which is the oracle's own; a logged decision
  for a key that is not inside the band must be ignored.
* The FP64 moment sums (E, E^2, E^4, M, M^2, M^4 per slot, eqs. 11-12) must
  equal the sums of the powers of the recorded series, and their means must
  match exact Boltzmann averages from full enumeration.
* Table 1's critical temperatures (section 5.1) lie below the q = 3
  mean-field bound of the pairs-once Hamiltonian, as the reading of eq. 2
  requires.
"""
import math
import os

import numpy as np
import pytest
import scipy.special as sp

from banded_cases import exchange_case, metropolis_case

HERE = os.path.dirname(os.path.abspath(__file__))


def test_metropolis_band_is_counted_and_replayed(orc):
    L, q, sigma = 24, 3, 0.5
    seed, T, (i, a, b, dE, u) = metropolis_case(orc, L, q, sigma)
    # the constructed margin is at rounding level
    assert abs(dE / T[0] + math.log(u)) < 1e-13
    own = orc.PT(L, q, sigma, T, seed, mode=0)
    own.sweep(1)
    st = own.stats()
    assert st["banded_met"] == 1
    runs = {}
    for dec in (0, 1):
        pt = orc.PT(L, q, sigma, T, seed, mode=0)
        pt.set_replay(met=[(0, 0, 0, dec)])
        pt.sweep(1)
        runs[dec] = (pt.spins(), pt.energies())
    assert not np.array_equal(runs[0][0][0], runs[1][0][0]), "the two decisions must lead to different states"
    # walkers other than 0 are unaffected
    np.testing.assert_array_equal(runs[0][0][1:], runs[1][0][1:])
    # the oracle's own decision is one of the two
    assert any(np.array_equal(own.spins(), runs[d][0]) for d in (0, 1))
    # both replayed trajectories keep a consistent tracked energy
    for d in (0, 1):
        pt = orc.PT(L, q, sigma, T, seed, mode=1)
        pt.set_replay(met=[(0, 0, 0, d)])
        pt.sweep(1)
        np.testing.assert_array_equal(pt.spins(), runs[d][0])
        assert pt.energies()[0] == pytest.approx(pt.energy_full(0), rel=1e-12)


def test_replayed_decision_outside_the_band_is_ignored(orc):
    L, q, sigma = 24, 3, 0.5
    seed, T, _ = metropolis_case(orc, L, q, sigma)
    ref = orc.PT(L, q, sigma, T, seed, mode=0)
    ref.set_replay(met=[(0, 0, 0, 1)])
    ref.run(3, 1)
    for dec in (0, 1):
        pt = orc.PT(L, q, sigma, T, seed, mode=0)
        # attempts 1..5 of walker 0 and attempt 0 of walker 1 are ordinary decisions
        pt.set_replay(met=[(0, 0, 0, 1)] + [(0, 0, t, dec) for t in range(1, 6)] + [(1, 0, 0, dec)],
                      ex=[(0, 0, 0, dec), (0, 1, 1, dec)])
        pt.run(3, 1)
        np.testing.assert_array_equal(pt.spins(), ref.spins())
        np.testing.assert_array_equal(pt.perm(), ref.perm())


def test_exchange_band_is_counted_and_replayed(orc):
    L, q, sigma = 24, 3, 0.5
    seed, T = exchange_case(orc, L, q, sigma)
    own = orc.PT(L, q, sigma, T, seed)
    own.exchange()
    assert own.stats()["banded_ex"] == 1
    perms = {}
    for dec in (0, 1):
        pt = orc.PT(L, q, sigma, T, seed)
        pt.set_replay(ex=[(0, 0, 0, dec)])
        pt.exchange()
        perms[dec] = list(pt.perm())
        assert pt.stats()["xchg_acc"][0] == dec
    assert perms == {0: [0, 1], 1: [1, 0]}
    assert list(own.perm()) in (perms[0], perms[1])


def test_moment_sums_equal_powers_of_the_series(orc):
    pt = orc.PT(16, 3, 0.5, [0.4, 0.9, 2.0], 5, mode=0, record=True)
    pt.run(400, 1)
    E, M = pt.series()
    st = pt.stats()
    assert st["samples"] == 400 == len(E)
    for name, x, p in [("sumE", E, 1), ("sumE2", E, 2), ("sumE4", E, 4), ("sumM", M, 1), ("sumM2", M, 2),
                       ("sumM4", M, 4)]:
        np.testing.assert_allclose(st[name], (x**p).sum(axis=0), rtol=1e-12, err_msg=name)


def _jackknife(x, nbins=40):
    b = np.array_split(np.asarray(x), nbins)
    m = np.array([a.mean() for a in b])
    return m.mean(), m.std(ddof=1) / math.sqrt(nbins)


def test_fourth_moments_against_full_enumeration(orc):
    """<E^4> and <M^4> per slot (the inputs of U_E and V_M, eqs. 11-12) from the
    oracle's accumulators within 4.5 sigma of exact enumeration at L = 6, q = 3."""
    from oracle.enumerate import boltzmann_moments

    L, q, sigma = 6, 3, 0.5
    T = np.array([0.5, 0.8, 1.3, 2.1])
    J = orc.jstar(L, sigma)
    exact, _ = boltzmann_moments(J, q, 1 / T)
    pt = orc.PT(L, q, sigma, T, 777, mode=0, record=True)
    pt.run(100_000, 1)
    E, M = pt.series()
    st = pt.stats()
    n = st["samples"]
    for k in range(len(T)):
        for name, acc, series in [("E4", "sumE4", E[:, k] ** 4), ("M4", "sumM4", M[:, k] ** 4),
                                  ("E2", "sumE2", E[:, k] ** 2), ("M2", "sumM2", M[:, k] ** 2)]:
            _, err = _jackknife(series)
            mean = st[acc][k] / n
            assert abs(mean - exact[k][name]) < 4.5 * err + 1e-12, (k, name, mean, exact[k][name], err)


def test_table1_critical_temperatures_below_mean_field_bound():
    """q = 3 mean field for H = -sum_{i<j} J*(|i-j|) delta(s_i, s_j): every site
    couples to the others with total 2 zeta(1 + sigma), and the mean-field
    transition of the 3-state Potts model sits at T_MF = J_tot / (4 ln 2).  Mean
    field overestimates T_c, so every printed T_c lies below T_MF, by a factor
    that falls as the interaction becomes shorter ranged (larger sigma); with
    pairs counted twice T_MF would double and the ratios would fall below 1/2."""
    rows = np.loadtxt(os.path.join(HERE, "golden", "table1_tc.txt"))
    sig, tc, err = rows[:, 0], rows[:, 1], rows[:, 2]
    tmf = 2 * sp.zeta(1 + sig) / (4 * math.log(2))
    ratio = tc / tmf
    assert np.all(tc + err < tmf)
    assert np.all(np.diff(ratio) < 0)
    assert ratio[0] > 0.95 and ratio[-1] > 0.7
    assert np.all(tc / (2 * tmf) < 0.5)

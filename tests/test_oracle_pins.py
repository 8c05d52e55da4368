"""Pins of the CPU oracle against values fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: library
routines (scipy, mpmath, rocRAND's host Philox), closed forms, brute force on
small inputs, published known-answer vectors, and exact special cases of the
dynamics.  None of these tests needs a GPU.
"""
import math
import os
import shutil
import subprocess

import mpmath
import numpy as np
import pytest
import scipy.special as sp

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- zeta, J*
@pytest.mark.parametrize("s", [1.05, 1.1, 1.3, 1.5, 1.8, 2.0])
@pytest.mark.parametrize("a", [1e-4, 0.01, 0.3, 0.5, 0.999, 1.0, 1.25, 1.999])
def test_hurwitz_zeta_against_libraries(orc, s, a):
    """eq. 7 against scipy.special.zeta and mpmath.zeta."""
    z = orc.hurwitz_zeta(s, a)
    assert z == pytest.approx(sp.zeta(s, a), rel=2e-15, abs=0)
    assert z == pytest.approx(float(mpmath.zeta(s, a)), rel=2e-15, abs=0)


@pytest.mark.parametrize("L,sigma", [(2, 0.5), (3, 0.3), (64, 0.5), (1024, 0.4), (16384, 0.3), (777, 0.9)])
def test_jstar_closed_forms(orc, L, sigma):
    """sum_{r=1}^{L-1} J*(r) = 2 zeta(s)(1 - L^-s) (every nonzero integer not a
    multiple of L appears once); J*(r) = J*(L-r); J*(0) = 0."""
    s = 1.0 + sigma
    J = orc.jstar(L, sigma)
    assert J[0] == 0.0
    assert math.fsum(J) == pytest.approx(2 * sp.zeta(s) * (1 - L ** -s), rel=5e-15)
    r = np.arange(1, L)
    # eq. 6 taken literally: near r -> L the term L^-s zeta(s, 1 - r/L) ~ 1 is the
    # product of a large zeta value and a small power, good to ~1e-13 relative.
    np.testing.assert_allclose(J[r], J[L - r], rtol=1e-13, atol=0)
    if L == 2:
        assert J[1] == pytest.approx(2 * (1 - 2 ** -s) * sp.zeta(s), rel=5e-16)


@pytest.mark.parametrize("L,sigma", [(8, 0.5), (64, 0.5), (64, 0.1), (100, 1.0)])
def test_jstar_brute_image_sum(orc, L, sigma):
    """eq. 5 summed image by image, |n| <= N, plus the integral bounds of the
    two tails: sum_{n>N} (nL +- r)^-s lies between int_{N+1}^inf and int_N^inf."""
    s = 1.0 + sigma
    J = orc.jstar(L, sigma)
    N = 200_000
    n = np.arange(1, N + 1, dtype=np.float64)
    for r in [1, 2, L // 3, L // 2, L - 1]:
        head = r ** -s + math.fsum((n * L + r) ** -s) + math.fsum((n * L - r) ** -s)

        def tail(lo, sign):  # int_lo^inf (xL + sign r)^-s dx
            return (lo * L + sign * r) ** (1 - s) / (L * (s - 1))

        low = head + tail(N + 1, 1) + tail(N + 1, -1)
        high = head + tail(N, 1) + tail(N, -1)
        assert low * (1 - 1e-13) <= J[r] <= high * (1 + 1e-13), (r, low, J[r], high)


def test_jstar_mpmath_direct(orc):
    """eq. 6 evaluated with mpmath at 30 digits."""
    mpmath.mp.dps = 30
    L, sigma = 1000, 0.37
    J = orc.jstar(L, sigma)
    s = mpmath.mpf(1) + mpmath.mpf(sigma)
    for r in [1, 17, 500, 999]:
        ref = mpmath.mpf(r) ** -s + mpmath.mpf(L) ** -s * (
            mpmath.zeta(s, 1 + mpmath.mpf(r) / L) + mpmath.zeta(s, 1 - mpmath.mpf(r) / L))
        assert J[r] == pytest.approx(float(ref), rel=4e-15)
    mpmath.mp.dps = 15


# ---------------------------------------------------------------- Philox
def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers(orc):
    for row in _kat():
        out = orc.philox4x32_10(row[0:4], row[4:6])
        assert [int(x) for x in out] == row[6:10]


def test_philox_against_rocrand_host_engine(orc, tmp_path):
    """rocRAND's philox4x32_10 engine (host path) at random counters and keys."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "rr"
    subprocess.check_call([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                           os.path.join(HERE, "rocrand_philox_ref.hip"), "-o", str(exe)],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(7)
    cases = rng.integers(0, 2**32, size=(64, 6), dtype=np.uint64)
    cases[:, 1] %= 2**30  # rocRAND takes words 0-1 as offset/4 in a 64-bit offset
    cases[:4, :] = [[0, 0, 0, 0, 0, 0], [5, 3, 7, 0, 1234, 0], [1023, 9999, 63, 0, 1234, 0],
                    [12, 1, 2, 2, 0xdeadbeef, 0x1]]
    text = "\n".join(" ".join("%x" % int(v) for v in c) for c in cases) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(x, 16) for x in line.split()] for line in out.strip().splitlines()]
    for c, g in zip(cases, got):
        ref = orc.philox4x32_10([int(v) for v in c[:4]], [int(v) for v in c[4:6]])
        assert [int(x) for x in ref] == g


# ---------------------------------------------------------------- energies
def test_energy_ordered_state_closed_form(orc):
    """All spins equal: E0 = -sum_{i<j} J*(j-i) = -L zeta(s) (1 - L^-s)."""
    for L, sigma in [(64, 0.5), (1000, 0.3), (7, 0.8)]:
        s = 1 + sigma
        J = orc.jstar(L, sigma)
        E0 = orc.energy(J, np.full(L, 2, np.uint8))
        # sequential sum of L(L-1)/2 terms: |error| <= npairs * 2^-53 * |E0|
        tol = 1.2 * (L * (L - 1) / 2) * 2.0**-53 + 1e-13
        assert E0 == pytest.approx(-L * sp.zeta(s) * (1 - L ** -s), rel=tol)


def test_energy_brute_pairs_and_mean_over_states(orc):
    """Pair enumeration against an explicit double loop, and the mean over all
    q^L states, which is E0/q exactly (each pair is equal with probability 1/q)."""
    from oracle.enumerate import energies, states

    L, q, sigma = 6, 3, 0.6
    J = orc.jstar(L, sigma)
    S = states(L, q)
    E = energies(J, S)
    idx = np.random.default_rng(1).integers(0, len(S), 50)
    for k in idx:
        ref = -sum(J[j - i] for i in range(L) for j in range(i + 1, L) if S[k, i] == S[k, j])
        assert orc.energy(J, S[k].astype(np.uint8)) == pytest.approx(ref, rel=1e-14, abs=1e-14)
        assert E[k] == pytest.approx(ref, rel=1e-14, abs=1e-14)
    E0 = -L * sp.zeta(1 + sigma) * (1 - L ** -(1 + sigma))
    assert E.mean() == pytest.approx(E0 / q, rel=1e-12)


def test_q2_potts_is_half_ising(orc):
    """delta(s_i,s_j) = (1 + sig_i sig_j)/2  =>  E_Potts = E_Ising/2 - (L/2) zeta(s)(1 - L^-s)."""
    rng = np.random.default_rng(3)
    for L, sigma in [(10, 0.5), (128, 0.2)]:
        J = orc.jstar(L, sigma)
        s = rng.integers(1, 3, L).astype(np.uint8)
        sig = np.where(s == 1, 1, -1).astype(np.int8)
        const = (L / 2) * sp.zeta(1 + sigma) * (1 - L ** -(1 + sigma))
        assert orc.energy(J, s) == pytest.approx(orc.energy_ising(J, sig) / 2 - const, rel=1e-12)


def test_magnetization_values(orc):
    assert orc.magnetization(3, np.ones(9, np.uint8)) == 1.0
    assert orc.magnetization(3, np.array([1, 2, 3] * 3, np.uint8)) == pytest.approx(0.0)
    assert orc.magnetization(4, np.array([1, 1, 2, 3], np.uint8)) == pytest.approx((4 * 2 / 4 - 1) / 3)


# ---------------------------------------------------------------- dynamics
def _philox_draws(orc, seed, L, q, w, n):
    """The attempt draws of the oracle's stream, restated from its definition:
    counter (t, n, w, 0), site = mulhi(o0, L), offset = 1 + mulhi(o1, q-1),
    u = ((o2 << 20 | o3 >> 12) + 1/2) 2^-52."""
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = []
    for t in range(L):
        o = [int(x) for x in orc.philox4x32_10([t, n, w, 0], key)]
        i = (o[0] * L) >> 32
        k = 1 + ((o[1] * (q - 1)) >> 32)
        u = (((o[2] << 20) | (o[3] >> 12)) + 0.5) * 2.0**-52
        out.append((i, k, u))
    return out


def test_infinite_temperature_accepts_every_proposal(orc):
    """beta = 0: x = ln u < 0 for every attempt, so each proposal is applied."""
    L, q, seed = 12, 4, 99
    pt = orc.PT(L, q, 0.5, [1e300, 1e300], seed, init=0, mode=0)
    s = pt.spins().astype(int)
    pt.sweep(3)
    for n in range(3):
        for w in range(2):
            for (i, k, _) in _philox_draws(orc, seed, L, q, w, n):
                s[w, i] = (s[w, i] - 1 + k) % q + 1
    np.testing.assert_array_equal(pt.spins(), s)
    st = pt.stats()
    assert (st["flip_acc"] == st["flip_att"]).all()


def test_initial_spins_from_stream(orc):
    L, q, seed = 33, 5, 2024
    pt = orc.PT(L, q, 0.5, [1.0, 2.0, 3.0], seed)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    ref = np.array([[1 + ((int(orc.philox4x32_10([j, 0, w, 2], key)[0]) * q) >> 32) for j in range(L)]
                    for w in range(3)])
    np.testing.assert_array_equal(pt.spins(), ref)
    assert (orc.PT(L, q, 0.5, [1.0], seed, init=1).spins() == 1).all()


def test_zero_temperature_ordered_start_rejects_everything(orc):
    """From the ordered state every flip raises E by sum J* > 0; at beta = 1e12
    no u in (0,1) accepts it."""
    pt = orc.PT(40, 3, 0.7, [1e-12, 1e-12], 5, init=1, mode=0)
    pt.sweep(5)
    assert (pt.spins() == 1).all()
    assert (pt.stats()["flip_acc"] == 0).all()


def test_q2_trajectory_matches_separately_written_ising(orc):
    """Potts q = 2 at beta follows the +-1 Ising path at beta/2 under the same draws."""
    L, sigma, seed = 48, 0.5, 77
    T = [0.7, 1.3]
    pt = orc.PT(L, 2, sigma, T, seed, init=0, mode=0)
    J = orc.jstar(L, sigma)
    s0 = pt.spins()
    E0 = pt.energies()
    const = (L / 2) * sp.zeta(1 + sigma) * (1 - L ** -(1 + sigma))
    pt.sweep(20)
    for w in range(2):
        sig = np.where(s0[w] == 1, 1, -1).astype(np.int8)
        sig, EI = orc.ising_sweeps(J, sig, 0.5 / T[w], seed, w, 0, 20, 2 * (E0[w] + const))
        np.testing.assert_array_equal(np.where(sig == 1, 1, 2), pt.spins()[w])
        assert pt.energies()[w] == pytest.approx(EI / 2 - const, rel=1e-10)


@pytest.mark.parametrize("q", [2, 3, 5])
def test_field_table_mode_matches_direct_mode(orc, q):
    """Two ways of evaluating the same energy difference give the same trajectory."""
    L, sigma, seed = 40, 0.45, 11
    T = [0.4, 0.8, 1.6, 3.2]
    a = orc.PT(L, q, sigma, T, seed, mode=0)
    b = orc.PT(L, q, sigma, T, seed, mode=1)
    for _ in range(30):
        a.run(1, 1); b.run(1, 1)
    np.testing.assert_array_equal(a.spins(), b.spins())
    np.testing.assert_array_equal(a.perm(), b.perm())
    np.testing.assert_allclose(a.energies(), b.energies(), rtol=1e-12)


def test_tracked_energy_equals_full_recomputation(orc):
    L, q, sigma = 64, 3, 0.5
    pt = orc.PT(L, q, sigma, [0.5, 1.0, 2.0, 4.0], 1234, mode=0)
    for _ in range(10):
        pt.run(20, 1)
        E = pt.energies()
        for w in range(4):
            assert E[w] == pytest.approx(pt.energy_full(w), rel=1e-10, abs=1e-10)


def test_exchange_equal_temperatures_always_swaps(orc):
    """Equal betas make the exponent of eq. 9 zero, so every attempt is accepted."""
    pt = orc.PT(16, 3, 0.5, [1.0, 1.0, 1.0, 1.0], 3)
    for _ in range(5):
        pt.exchange()
    st = pt.stats()
    assert (st["xchg_acc"] == st["xchg_att"]).all()
    # two stages per step: pairs (0,1),(2,3) then (1,2)
    assert list(st["xchg_att"]) == [5, 5, 5]


def test_exchange_rule_direction(orc):
    """A cold slot holding the higher energy always swaps (exponent > 0); a
    cold slot holding the ordered state and a hot one a disordered state with
    a large beta gap essentially never does."""
    L, q, sigma = 32, 3, 0.5
    pt = orc.PT(L, q, sigma, [0.1, 10.0], 5, init=0)
    s = np.ones((2, L), np.uint8)
    s[0] = np.array([1, 2, 3] * 10 + [1, 2], np.uint8)  # walker 0 (cold slot) disordered
    pt.set_spins(s)
    pt.exchange()
    assert list(pt.perm()) == [1, 0]
    pt.exchange()  # now the cold slot holds the ordered walker
    assert list(pt.perm()) == [1, 0]


# ---------------------------------------------------------------- equilibrium
def _jackknife(x, nbins=40):
    b = np.array_split(np.asarray(x), nbins)
    m = np.array([a.mean() for a in b])
    return m.mean(), m.std(ddof=1) / math.sqrt(nbins)


@pytest.mark.parametrize("mode", [0, 1])
def test_equilibrium_against_full_enumeration(orc, mode):
    """L = 6, q = 3: MC moments and exchange rates within 4.5 sigma of the exact values."""
    from oracle.enumerate import boltzmann_moments, exchange_rates

    L, q, sigma = 6, 3, 0.5
    T = np.array([0.5, 0.8, 1.3, 2.1])
    J = orc.jstar(L, sigma)
    exact, _ = boltzmann_moments(J, q, 1 / T)
    rates = exchange_rates(J, q, 1 / T)
    pt = orc.PT(L, q, sigma, T, 4321, mode=mode, record=True)
    pt.run(2000, 1)
    E0, M0 = pt.series()
    pt = orc.PT(L, q, sigma, T, 4321, mode=mode, record=True)
    pt.run(120_000, 1)
    E, M = pt.series()
    E, M = E[2000:], M[2000:]
    for k in range(len(T)):
        for name, series in [("E", E[:, k]), ("E2", E[:, k] ** 2), ("M", M[:, k]), ("M2", M[:, k] ** 2)]:
            mean, err = _jackknife(series)
            assert abs(mean - exact[k][name]) < 4.5 * err + 1e-12, (k, name, mean, exact[k][name], err)
    st = pt.stats()
    acc = st["xchg_acc"] / st["xchg_att"]
    for k in range(len(T) - 1):
        p = rates[k]
        err = math.sqrt(p * (1 - p) / st["xchg_att"][k]) * 3  # autocorrelation allowance
        assert abs(acc[k] - p) < 4.5 * err, (k, acc[k], p)


def test_walker_offset_follows_the_larger_run(orc):
    """A one-walker object with wbase = w reproduces walker w of a larger run
    (same temperature, no exchange)."""
    T = [0.5, 0.9, 1.4, 2.2]
    big = orc.PT(30, 3, 0.6, T, 9, mode=0)
    big.sweep(6)
    for w in (1, 3):
        one = orc.PT(30, 3, 0.6, [T[w]], 9, mode=0, wbase=w)
        one.sweep(6)
        np.testing.assert_array_equal(one.spins()[0], big.spins()[w])

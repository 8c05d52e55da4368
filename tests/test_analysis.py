"""Host-side thermodynamic analysis (paper section 5.1, eqs. 11-12): cumulants,
jackknife errors, Binder crossings, power-law extrapolation.  CPU only."""
import math

import numpy as np
import pytest

from paper_1308_5426_amd import analysis as an


def test_cumulant_limits():
    # constant energy: <E^4> = <E^2>^2 -> U_E = 1; fully ordered: M = 1 -> V_M = 2/3
    assert an.energy_cumulant(4.0, 16.0) == 1.0
    assert an.binder_cumulant(1.0, 1.0) == pytest.approx(2.0 / 3.0)
    # symmetric two-point M = +-m: <M^4> = <M^2>^2 -> 2/3 as well; Gaussian M: <M^4> = 3<M^2>^2 -> 0
    assert an.binder_cumulant(0.25, 0.0625) == pytest.approx(2.0 / 3.0)
    assert an.binder_cumulant(2.0, 12.0) == pytest.approx(0.0)


def test_jackknife_gaussian_mean_and_error():
    rng = np.random.default_rng(0)
    x = rng.normal(3.0, 2.0, size=(40000, 1))
    m, e = an.jackknife({"x": x}, lambda b: b["x"], nbins=40)
    assert abs(m[0] - 3.0) < 4 * 2.0 / math.sqrt(40000)
    assert e[0] == pytest.approx(2.0 / math.sqrt(40000), rel=0.35)


def test_jackknife_removes_ratio_bias():
    """Jackknife of a ratio of means is less biased than the plain ratio."""
    rng = np.random.default_rng(1)
    bias_plain, bias_jk = [], []
    for _ in range(200):
        x = rng.exponential(1.0, size=(64, 1)) + 0.5
        plain = 1.0 / x.mean()
        jk, _ = an.jackknife({"x": x}, lambda b: 1.0 / b["x"], nbins=64)
        bias_plain.append(plain - 1 / 1.5)
        bias_jk.append(jk[0] - 1 / 1.5)
    assert abs(np.mean(bias_jk)) < abs(np.mean(bias_plain))


def test_crossing_of_synthetic_curves():
    T = np.linspace(1.0, 2.0, 41)
    Tc = 1.4375
    v1 = 0.3 - 0.2 * np.tanh(3.0 * (T - Tc))
    v2 = 0.3 - 0.2 * np.tanh(7.0 * (T - Tc))
    assert an.crossing(T, v1, T, v2) == pytest.approx(Tc, abs=2e-3)
    est, pairs = an.binder_crossings({64: (T, v1), 128: (T, v2), 256: (T, 0.3 - 0.2 * np.tanh(15 * (T - Tc)))})
    assert est == pytest.approx(Tc, abs=3e-3)
    assert len(pairs) == 3
    assert an.crossing(T, v1, T, v1 + 1.0) is None


def test_power_law_fit_recovers_parameters():
    L = np.array([1024, 1536, 2048, 3072, 4096, 5120], float)
    U = 1.022 + 3.5 * L ** -0.8
    (u, a, b), err = an.power_law_fit(L, U)
    assert u == pytest.approx(1.022, abs=1e-8)
    assert a == pytest.approx(3.5, rel=1e-6)
    assert b == pytest.approx(0.8, rel=1e-6)


def test_cumulants_against_enumeration(orc):
    """Oracle MC series at L = 6, q = 3: U_E and V_M per slot within 5 jackknife
    errors of the values from full enumeration."""
    from oracle.enumerate import boltzmann_moments

    L, q, sigma = 6, 3, 0.5
    T = np.array([0.5, 1.0, 2.0])
    J = orc.jstar(L, sigma)
    exact, _ = boltzmann_moments(J, q, 1 / T)
    pt = orc.PT(L, q, sigma, T, 99, mode=0, record=True)
    pt.run(60000, 1)
    E, M = pt.series()
    E, M = E[1000:], M[1000:]
    (ue, uerr), (vm, verr) = an.cumulants_with_errors(E, M, nbins=40)
    for k in range(len(T)):
        ue_x = exact[k]["E4"] / exact[k]["E2"] ** 2
        vm_x = 1 - exact[k]["M4"] / (3 * exact[k]["M2"] ** 2)
        assert abs(ue[k] - ue_x) < 5 * uerr[k] + 1e-12, (k, ue[k], ue_x, uerr[k])
        assert abs(vm[k] - vm_x) < 5 * verr[k] + 1e-12, (k, vm[k], vm_x, verr[k])
    st = pt.stats()
    m = an.from_sums(dict(samples=st["samples"], **{("sum" + k): st["sum" + k] for k in
                                                  ("E", "E2", "E4", "M", "M2", "M4")}))
    np.testing.assert_allclose(m["E"], E.mean(axis=0), rtol=0.05)

"""The Binder-cumulant driver (section 5.1, eq. 12) on a small run: V_M per
temperature with jackknife errors, ordered limit 2/3 at low T, and a value
well below it at high T."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def binder():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1308_5426_amd import binder as b

    return b


def test_binder_curve_limits(binder):
    T = np.linspace(0.2, 6.0, 16)
    V, dV, xr, _ = binder.binder_curve(64, 0.6, T, therm=300, prod=800, blocks=4, seed=7)
    assert V.shape == (16,) and dV.shape == (16,)
    assert np.all(np.isfinite(V)) and np.all(dV >= 0.0)
    # ordered phase: M = 1 at every sample, so <M^4> = <M^2>^2 and V_M = 2/3
    assert abs(V[0] - 2.0 / 3.0) < 1e-3
    assert V[-1] < V[0] - 0.05
    assert np.all((xr >= 0.0) & (xr <= 1.0))


def test_binder_main_prints_crossings(binder, capsys):
    binder.main(["--sigma", "0.6", "--sizes", "32,64", "--tmin", "0.8", "--tmax", "2.5", "--replicas", "8",
                 "--therm", "200", "--prod", "400", "--blocks", "4"])
    import json

    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["Tc_table1"] == 1.4125
    assert set(out["curves"]) == {"32", "64"}


def test_binder_energy_cumulant_and_fit(binder, capsys):
    binder.main(["--sigma", "0.5", "--sizes", "32,48,64", "--tmin", "1.0", "--tmax", "2.4", "--replicas", "8",
                 "--therm", "200", "--prod", "400", "--blocks", "4", "--energy-cumulant"])
    import json

    out = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert out["U_E_inf_table2"] == 1.022
    for L in ("32", "48", "64"):
        u, du, t = out["curves"][L]["U_E_max"]
        assert u >= 1.0 and du >= 0.0 and 1.0 <= t <= 2.4  # <E^4> >= <E^2>^2 (Jensen)
    assert "U_E_inf" in out


def test_binder_curve_equals_oracle_moments(binder):
    """The cumulants the driver forms from the GPU's FP64 moment sums (V_M,
    eq. 12; U_E, eq. 11) equal those formed the same way from the oracle's sums
    over the same production blocks on the same streams."""
    import oracle
    from paper_1308_5426_amd.analysis import binder_cumulant, energy_cumulant, jackknife

    L, sigma, seed, therm, prod, blocks = 32, 0.6, 7, 60, 120, 4
    T = np.linspace(0.8, 2.5, 8)
    V, dV, xr, _, U, dU = binder.binder_curve(L, sigma, T, therm, prod, blocks, seed, with_energy=True)
    ref = oracle.PT(L, 3, sigma, T, seed, mode=0)
    ref.run(therm, 1)
    s0 = s_therm = ref.stats()
    per = prod // blocks
    blk = {k: [] for k in ("M2", "M4", "E2", "E4")}
    for _ in range(blocks):
        ref.run(per, 1)
        s1 = ref.stats()
        for k in blk:  # the block's sums: differences of the oracle's running sums
            blk[k].append((s1["sum" + k] - s0["sum" + k]) / per)
        s0 = s1
    assert s1["banded_met"] == 0 and s1["banded_ex"] == 0
    Vr, dVr = jackknife({"M2": np.array(blk["M2"]), "M4": np.array(blk["M4"])},
                        lambda m: binder_cumulant(m["M2"], m["M4"]), nbins=blocks)
    Ur, dUr = jackknife({"E2": np.array(blk["E2"]), "E4": np.array(blk["E4"])},
                        lambda m: energy_cumulant(m["E2"], m["E4"]), nbins=blocks)
    np.testing.assert_allclose(V, Vr, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(dV, dVr, rtol=1e-6, atol=1e-12)
    np.testing.assert_allclose(U, Ur, rtol=1e-9)
    np.testing.assert_allclose(dU, dUr, rtol=1e-6, atol=1e-12)
    acc, att = s1["xchg_acc"] - s_therm["xchg_acc"], s1["xchg_att"] - s_therm["xchg_att"]
    np.testing.assert_allclose(xr, acc / np.maximum(att, 1))

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

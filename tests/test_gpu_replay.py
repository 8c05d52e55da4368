"""The banded-replay protocol on the GPU, the exchange schedule of pt_run, and
the phase counters.  Marked gpu; every case goes through the C ABI.

A decision placed exactly at its threshold (tests/banded_cases.py) must reach
the FP64 recheck, be logged as a banded event under the oracle's key, and,
once the oracle adopts the logged decision, leave identical trajectories.
"""
import numpy as np
import pytest

from banded_cases import exchange_case, metropolis_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_5426_amd as p

    p.load_library()
    return p


def _replay(ref, events):
    ref.set_replay(met=[(a, b, c, d) for (k, a, b, c, d, _) in events if k == 0],
                   ex=[(a, b, c, d) for (k, a, b, c, d, _) in events if k == 1])


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_metropolis_band_logged_and_replayed(pkg, orc, precision):
    L, q, sigma = 24, 3, 0.5
    seed, T, _ = metropolis_case(orc, L, q, sigma)
    print(f"[replay] metropolis band seed={seed} precision={precision}", flush=True)
    sim = pkg.Simulation(L, q, sigma, T, seed, precision=precision)
    sim.run(4, 1)
    ev = sim.events()
    obs = sim.observables()
    assert any(k == 0 and (a, b, c) == (0, 0, 0) for (k, a, b, c, d, x) in ev), ev
    assert all(abs(x) <= pkg.BAND for (*_, x) in ev)
    assert obs["n_banded"] >= 1
    assert obs["n_recheck"] >= 1  # the threshold decision went through the FP64 recheck
    ref = orc.PT(L, q, sigma, T, seed, mode=0)
    _replay(ref, ev)
    ref.run(4, 1)
    s, p = sim.spins()
    np.testing.assert_array_equal(s, ref.spins())
    np.testing.assert_array_equal(p, ref.perm())
    np.testing.assert_allclose(obs["E"], ref.energies()[ref.perm()], rtol=1e-6 if precision else 1e-12)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_exchange_band_logged_and_replayed(pkg, orc, precision):
    L, q, sigma = 24, 3, 0.5
    seed, T = exchange_case(orc, L, q, sigma)
    print(f"[replay] exchange band seed={seed} precision={precision}", flush=True)
    sim = pkg.Simulation(L, q, sigma, T, seed, precision=precision)
    sim.exchange()
    sim.run(5, 1)
    ev = sim.events()
    assert any(k == 1 and (a, b, c) == (0, 0, 0) for (k, a, b, c, d, x) in ev), ev
    ref = orc.PT(L, q, sigma, T, seed, mode=0)
    _replay(ref, ev)
    ref.exchange()
    ref.run(5, 1)
    s, p = sim.spins()
    np.testing.assert_array_equal(s, ref.spins())
    np.testing.assert_array_equal(p, ref.perm())
    obs = sim.observables()
    st = ref.stats()
    np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
    np.testing.assert_array_equal(obs["xchg_att"], st["xchg_att"])


def _pair(pkg, orc, L, q, sigma, T, seed, **kw):
    return (pkg.Simulation(L, q, sigma, T, seed, **kw), orc.PT(L, q, sigma, T, seed, mode=0))


def _same(sim, ref):
    s, p = sim.spins()
    np.testing.assert_array_equal(s, ref.spins())
    np.testing.assert_array_equal(p, ref.perm())
    obs = sim.observables()
    st = ref.stats()
    np.testing.assert_array_equal(obs["xchg_att"], st["xchg_att"])
    np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])


@pytest.mark.parametrize("chunk,every,n", [(4, 7, 30), (5, 5, 23), (3, 1, 10), (16, 40, 90)])
def test_run_schedule_independent_of_launch_size(pkg, orc, chunk, every, n):
    """An exchange step after sweeps every, 2 every, ... of the call, also when
    `every` exceeds the sweeps of one launch (max_sweeps_per_launch = chunk)."""
    from workloads import geometric_ladder

    T = geometric_ladder(0.4, 2.5, 6)
    print(f"[schedule] chunk={chunk} every={every} n={n}", flush=True)
    sim, ref = _pair(pkg, orc, 40, 3, 0.5, T, 31, max_sweeps_per_launch=chunk)
    sim.run(n, every)
    _replay(ref, sim.events())
    ref.run(n, every)
    _same(sim, ref)
    assert sim.observables()["exchange_steps"] == n // every


def test_run_after_partial_period(pkg, orc):
    """pt_run after pt_sweep(k), k not a multiple of every: the schedule restarts with the call."""
    from workloads import geometric_ladder

    T = geometric_ladder(0.4, 2.5, 5)
    sim, ref = _pair(pkg, orc, 50, 4, 0.6, T, 8, max_sweeps_per_launch=6)
    sim.sweep(3)
    sim.run(17, 4)
    sim.run(9, 2)
    _replay(ref, sim.events())
    ref.sweep(3)
    ref.run(17, 4)
    ref.run(9, 2)
    _same(sim, ref)
    assert sim.observables()["exchange_steps"] == 17 // 4 + 9 // 2


def test_phase_counters(pkg, orc):
    """Per-walker counters: every window counted, flips equal to the accepts,
    the timed phases within the walker's total, nothing without profiling."""
    from workloads import geometric_ladder

    L, R, n = 300, 6, 12
    T = geometric_ladder(0.3, 3.0, R)
    sim = pkg.Simulation(L, 3, 0.5, T, 4, profile=True)
    sim.run(n, 1)
    ph = sim.phase_counters()
    obs = sim.observables()
    assert (ph["windows"] == n * ((L + 63) // 64)).all()
    assert ph["flips"].sum() == obs["flip_acc"].sum()
    assert (ph["flushes"] <= ph["windows"]).all()
    assert (ph["iters"] >= ph["windows"]).all()
    timed = sum(ph[k] for k in ("draw", "chain", "flush", "record", "exchange"))
    assert (timed <= ph["total"]).all() and (timed >= 0.5 * ph["total"]).all()
    assert (ph["chain"] > 0).all()
    # the chain's steps are timed inside its own phase, every one at least once
    steps = [ph[k] for k in ("chain_guess", "chain_correct", "chain_check", "chain_resolve", "chain_redo",
                             "chain_sync")]
    assert (sum(steps) <= ph["chain"]).all()
    assert all((x > 0).all() for x in steps[:3])
    plain = pkg.Simulation(L, 3, 0.5, T, 4)
    with pytest.raises(pkg.PTError):
        plain.phase_counters()
    # profiling changes no decision
    plain.run(n, 1)
    np.testing.assert_array_equal(plain.spins()[0], sim.spins()[0])

"""pt_run_static, the entry point that allocates nothing, against the context
path it folds together (pt_init + pt_run + pt_observables + pt_get_spins) on
the same inputs: identical spins, slot permutation, counters and moments.  Two
calls in a row on the one static buffer, the second smaller than the first,
so that state left by a call cannot leak into the next."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pkg():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1308_5426_amd as p

    p.load_library()
    return p


def _ladder(tmin, tmax, R):
    from workloads import geometric_ladder

    return geometric_ladder(tmin, tmax, R)


def _context_path(pkg, L, q, sigma, T, seed, n, every, prec, init):
    sim = pkg.Simulation(L, q, sigma, T, seed, precision=prec, init=init)
    sim.run(n, every)
    obs = sim.observables()
    spins, perm = sim.spins()
    sim.close()
    return obs, spins, perm


def _compare(a, b):
    for k in ("flip_att", "flip_acc", "xchg_att", "xchg_acc", "perm"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)
    for k in ("sweeps", "exchange_steps", "samples", "n_recheck", "n_banded", "n_exact_energy", "n_refresh"):
        assert a[k] == b[k], k
    for k in ("E", "M", "sumE", "sumE2", "sumE4", "sumM", "sumM2", "sumM4"):
        np.testing.assert_allclose(a[k], b[k], rtol=1e-12, atol=0, err_msg=k)


# the 1024-site, 64-replica workload's shape first, then a smaller ragged one
CASES = [
    dict(L=1024, q=3, sigma=0.4, T=_ladder(0.3, 3.0, 64), seed=1234, n=24, every=1, prec=0, init=0),
    dict(L=100, q=5, sigma=0.7, T=_ladder(0.5, 2.0, 7), seed=77, n=33, every=2, prec=1, init=1),
]


def test_static_equals_context_path_two_calls(pkg):
    for c in CASES:
        print(f"[no-alloc] L={c['L']} q={c['q']} R={len(c['T'])} sweeps={c['n']} every={c['every']} "
              f"prec={c['prec']}", flush=True)
        obs_s, spins_s, perm_s = pkg.run_static(c["L"], c["q"], c["sigma"], c["T"], c["seed"], c["n"], c["every"],
                                                precision=c["prec"], init=c["init"])
        obs_c, spins_c, perm_c = _context_path(pkg, c["L"], c["q"], c["sigma"], c["T"], c["seed"], c["n"],
                                               c["every"], c["prec"], c["init"])
        np.testing.assert_array_equal(spins_s, spins_c)
        np.testing.assert_array_equal(perm_s, perm_c)
        _compare(obs_s, obs_c)
        assert obs_s["flip_acc"].sum() > 0


def test_static_refuses_state_beyond_its_buffer(pkg):
    # 128 replicas of 65535 sites in FP64: far beyond the static buffer; refused on the host
    with pytest.raises(pkg.PTError) as ei:
        pkg.run_static(65535, 16, 0.5, _ladder(0.5, 2.0, 128), 1, 1, 1)
    assert ei.value.status == pkg.PT_EINVAL
    assert "static buffer" in str(ei.value)

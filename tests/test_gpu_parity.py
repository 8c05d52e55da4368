"""Parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Trajectory parity: on the same Philox streams the GPU and the oracle must
produce identical spins and slot permutations after every step.  The only
admissible differences are decisions whose FP64 margin lies inside the 1e-9
band; the GPU logs those and the oracle adopts a logged decision only where
its own margin is also inside the band (banded replay).  Energies agree to
1e-12 relative (FP64 table) or within the rigorous bound the GPU carries
(FP32 table).
"""
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


def _replay(ref, events):
    ref.set_replay(met=[(a, b, c, d) for (k, a, b, c, d, _) in events if k == 0],
                   ex=[(a, b, c, d) for (k, a, b, c, d, _) in events if k == 1])


def _ladder(tmin, tmax, R):
    from workloads import geometric_ladder

    return geometric_ladder(tmin, tmax, R)


def run_pair(pkg, orc, L, q, sigma, T, seed, nsw, every=1, precision=0, init=0, threads=0,
             mode=0, steps=1, unfused=False, series=False, refresh_every=0):
    """Run GPU and oracle side by side in `steps` chunks; compare after each."""
    print(f"[parity] L={L} q={q} sigma={sigma} R={len(T)} sweeps={nsw} every={every} prec={precision} "
          f"init={init} threads={threads} unfused={unfused}", flush=True)
    sim = pkg.Simulation(L, q, sigma, T, seed, precision=precision, init=init, threads=threads,
                         series_capacity=nsw if series else 0, refresh_every=refresh_every)
    ref = orc.PT(L, q, sigma, T, seed, init=init, mode=mode, threads=8, record=series)
    s0, p0 = sim.spins()
    np.testing.assert_array_equal(s0, ref.spins())
    per = nsw // steps
    for st in range(steps):
        if unfused:
            for _ in range(per):
                sim.sweep(1)
                if every:
                    sim.exchange()
        else:
            sim.run(per, every)
        ev = sim.events()
        _replay(ref, ev)
        ref.run(per, every)
        s, p = sim.spins()
        bad = np.argwhere(s != ref.spins())
        assert bad.size == 0, f"step {st}: spins differ at {bad[:5]}"
        np.testing.assert_array_equal(p, ref.perm())
    return sim, ref


def _cmp_energy(sim, ref, rtol):
    obs = sim.observables()
    E_ref = ref.energies()[ref.perm()]
    np.testing.assert_allclose(obs["E"], E_ref, rtol=rtol, atol=rtol * 10)
    return obs


# ---------------------------------------------------------------- a1, a2, a3
@pytest.mark.parametrize("L,sigma", [(2, 0.5), (3, 0.2), (64, 0.5), (1000, 0.37), (1024, 0.4), (16384, 0.3),
                                     (4097, 1.0), (128, 0.1)])
def test_jstar_kernel_matches_oracle(pkg, orc, L, sigma):
    sim = pkg.Simulation(L, 2, sigma, [1.0], 1)
    J = sim.jstar()
    ref = orc.jstar(L, sigma)
    assert J[0] == 0.0
    np.testing.assert_allclose(J[1:], ref[1:], rtol=1e-12, atol=0)


@pytest.mark.parametrize("init", [0, 1])
@pytest.mark.parametrize("L,q,R", [(64, 3, 16), (100, 7, 3), (1024, 3, 64), (37, 16, 5)])
def test_initial_state_matches_oracle(pkg, orc, L, q, R, init):
    T = _ladder(0.3, 3.0, R)
    sim = pkg.Simulation(L, q, 0.5, T, 1234, init=init)
    ref = orc.PT(L, q, 0.5, T, 1234, init=init)
    s, p = sim.spins()
    np.testing.assert_array_equal(s, ref.spins())
    np.testing.assert_array_equal(p, np.arange(R))
    obs = sim.observables()
    np.testing.assert_allclose(obs["E"], ref.energies(), rtol=1e-12)
    M_ref = [orc.magnetization(q, ref.spins()[w]) for w in range(R)]
    np.testing.assert_allclose(obs["M"], M_ref, rtol=1e-14)


# ---------------------------------------------------------------- a4-a7
def test_small_config_trajectory_fp64(pkg, orc):
    """L = 64, q = 3, sigma = 0.5, 16 replicas geometric in [0.3, 3], seed 1234,
    2000 sweeps with an exchange step after each; E and M recorded per slot."""
    T = _ladder(0.3, 3.0, 16)
    sim, ref = run_pair(pkg, orc, 64, 3, 0.5, T, 1234, 2000, 1, precision=0, steps=4, series=True)
    obs = _cmp_energy(sim, ref, 1e-12)
    Eg, Mg = sim.series()
    Er, Mr = ref.series()
    assert Eg.shape == Er.shape == (2000, 16)
    np.testing.assert_allclose(Eg, Er, rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(Mg, Mr, rtol=1e-14, atol=1e-14)
    st = ref.stats()
    np.testing.assert_array_equal(obs["flip_att"], st["flip_att"])
    np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
    np.testing.assert_array_equal(obs["xchg_att"], st["xchg_att"])
    np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
    for k in ("sumE", "sumE2", "sumE4"):
        np.testing.assert_allclose(obs[k], st[k], rtol=1e-11)
    for k in ("sumM", "sumM2", "sumM4"):
        np.testing.assert_allclose(obs[k], st[k], rtol=1e-12)


@pytest.mark.parametrize("precision", [1, 2])
def test_small_config_trajectory_fp32_int32(pkg, orc, precision):
    """Same workload with the FP32 field table and with the int32 table of
    quantised couplings: decisions are FP64-exact through the rechecks, so the
    trajectory is identical; energies within 1e-6 relative.  The FP32 table is
    refreshed when its drift reaches the cap; the int32 table never drifts."""
    T = _ladder(0.3, 3.0, 16)
    sim, ref = run_pair(pkg, orc, 64, 3, 0.5, T, 1234, 2000, 1, precision=precision, steps=2)
    obs = sim.observables()
    E_ref = ref.energies()[ref.perm()]
    np.testing.assert_allclose(obs["E"], E_ref, rtol=1e-6)
    print(f"[parity] C1 prec={precision}: {obs['n_recheck']} rechecks, {obs['n_refresh']} refreshes", flush=True)
    if precision == 1:
        assert obs["n_refresh"] > 0  # the hot walkers' table drift reached its cap
    else:
        assert obs["n_refresh"] == 0


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_fused_equals_unfused(pkg, orc, precision):
    """Persistent launch with device-side exchange vs one launch per sweep and
    per exchange step."""
    T = _ladder(0.4, 2.5, 8)
    run_pair(pkg, orc, 96, 4, 0.6, T, 7, 60, 1, precision=precision, unfused=True, steps=2)
    run_pair(pkg, orc, 96, 4, 0.6, T, 7, 60, 3, precision=precision, steps=3)


@pytest.mark.parametrize("L,q,threads", [(100, 2, 64), (1000, 5, 256), (1000, 5, 192), (1000, 5, 64),
                                         (257, 16, 128), (2, 2, 64), (3, 3, 64), (1000, 3, 256),
                                         (1000, 4, 128), (100, 3, 64), (2500, 3, 256)])
def test_tiles_and_ragged_sizes(pkg, orc, L, q, threads):
    T = _ladder(0.2, 3.0, 6)
    run_pair(pkg, orc, L, q, 0.45, T, 99, 20, 1, threads=threads, steps=2, mode=1 if L >= 1000 else 0)


@pytest.mark.parametrize("L,q,threads", [(100, 2, 64), (1000, 5, 256), (257, 16, 128), (2, 2, 64), (1000, 7, 192),
                                         (2500, 3, 256)])
def test_tiles_and_ragged_sizes_int32(pkg, orc, L, q, threads):
    """The int32 table across tile shapes, ragged sizes and the three flush
    forms (four rows, eight rows, row by row)."""
    T = _ladder(0.2, 3.0, 6)
    run_pair(pkg, orc, L, q, 0.45, T, 99, 20, 1, precision=2, threads=threads, steps=2, mode=1 if L >= 1000 else 0)


def test_single_replica(pkg, orc):
    run_pair(pkg, orc, 77, 3, 0.5, [1.1], 5, 30, 1, steps=1)


def test_ordered_start_and_extreme_temperatures(pkg, orc):
    # T tiny: nothing accepted from the ordered state; T huge: every proposal accepted
    sim, ref = run_pair(pkg, orc, 80, 3, 0.7, [1e-9, 1e-9], 3, 10, 1, init=1)
    obs = sim.observables()
    assert (obs["flip_acc"] == 0).all()
    sim, ref = run_pair(pkg, orc, 80, 3, 0.7, [1e200, 1e200], 3, 10, 0, init=1)
    obs = sim.observables()
    assert (obs["flip_acc"] == obs["flip_att"]).all()


def test_medium_config_sampled(pkg, orc):
    """L = 1024, q = 3, sigma = 0.4, 64 replicas geometric in [0.3, 3] at its real
    size and launch shape: FP32 table for 40 sweeps (past the hot walkers'
    drift-driven refreshes, with near-threshold FP64 rechecks), FP64 table for
    12 sweeps."""
    T = _ladder(0.3, 3.0, 64)
    for prec, nsw in ((1, 40), (2, 40), (0, 12)):
        sim, ref = run_pair(pkg, orc, 1024, 3, 0.4, T, 1234, nsw, 1, precision=prec, mode=1, steps=2)
        obs = sim.observables()
        E_ref = ref.energies()[ref.perm()]
        np.testing.assert_allclose(obs["E"], E_ref, rtol=1e-6 if prec else 1e-11)
        st = ref.stats()
        np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
        np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
        print(f"[parity] C2 prec={prec}: {obs['n_recheck']} rechecks, {obs['n_refresh']} refreshes", flush=True)
        if prec == 1:
            assert obs["n_recheck"] > 0
            assert obs["n_refresh"] > 0
        if prec == 2:
            assert obs["n_refresh"] == 0


def test_checkpoint_resume(pkg, orc):
    T = _ladder(0.3, 3.0, 8)
    a = pkg.Simulation(50, 3, 0.5, T, 21)
    a.run(30, 1)
    blob = a.save()
    a.run(30, 1)
    b = pkg.Simulation.load(blob)
    b.run(30, 1)
    sa, pa = a.spins()
    sb, pb = b.spins()
    np.testing.assert_array_equal(sa, sb)
    np.testing.assert_array_equal(pa, pb)
    oa, ob = a.observables(), b.observables()
    np.testing.assert_array_equal(oa["flip_acc"], ob["flip_acc"])
    np.testing.assert_allclose(oa["E"], ob["E"], rtol=1e-12)


def test_invalid_arguments(pkg):
    T = [1.0, 2.0]
    for args in [(1, 3, 0.5, T), (10, 1, 0.5, T), (10, 17, 0.5, T), (10, 3, 0.0, T), (10, 3, -1.0, T),
                 (10, 3, 0.5, [2.0, 1.0]), (10, 3, 0.5, [1.0, float("nan")]), (10, 3, 0.5, [0.0, 1.0])]:
        with pytest.raises(pkg.PTError) as ei:
            pkg.Simulation(*args, 1)
        assert ei.value.status == pkg.PT_EINVAL


@pytest.mark.parametrize("placement,precision", [(0, 1), (2, 1), (3, 1), (0, 2), (2, 0)])
def test_large_config_all_walkers(pkg, orc, placement, precision):
    """L = 16384, q = 5, sigma = 0.3, 128 replicas geometric in [0.2, 2.5], ordered
    start, FP32 form, at the real launch shape: three sweeps of every walker with
    the fused exchange step after each, against the oracle on all walkers, with
    the field table in HBM (the automatic choice: it does not fit in LDS) and
    with direct sums and no table; also the int32 and FP64 tables in HBM."""
    from workloads import large

    inst = large()
    nsw = 3
    print(f"[parity] large L={inst.L} q={inst.q} R={inst.R} placement={placement} precision={precision} "
          f"sweeps={nsw}", flush=True)
    sim = pkg.Simulation(inst.L, inst.q, inst.sigma, inst.T, inst.seed, precision=precision, init=inst.init,
                         placement=placement)
    assert sim.plan()["placement"] == (placement or pkg.PLACE_HBM)
    sim.run(nsw, 1)
    s, p = sim.spins()
    obs = sim.observables()
    ev = sim.events()
    ref = orc.PT(inst.L, inst.q, inst.sigma, inst.T, inst.seed, init=inst.init, mode=0, threads=16)
    _replay(ref, ev)
    ref.run(nsw, 1)
    np.testing.assert_array_equal(s, ref.spins())
    np.testing.assert_array_equal(p, ref.perm())
    st = ref.stats()
    np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
    np.testing.assert_array_equal(obs["xchg_att"], st["xchg_att"])
    np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
    # direct sums: the oracle's initial energy is a sequential sum of L(L-1)/2
    # terms, whose rounding error is bounded by (L^2/2) 2^-53 |E| (about 1.5e-8
    # here); FP32 table: energy changes summed from the FP32 couplings, 1e-6
    rtol = inst.L * inst.L / 2 * 2.0**-53 if (placement == 3 or precision == 0) else 1e-6
    np.testing.assert_allclose(obs["E"], ref.energies()[ref.perm()], rtol=rtol)


@pytest.mark.parametrize("precision", [0, 2])
@pytest.mark.parametrize("L,q", [(256, 2), (300, 3), (1000, 4), (1024, 3)])
def test_overlapped_sweep_matches_oracle(pkg, orc, L, q, precision):
    """The overlapped sweep (512 threads: chain of window s beside the flush of
    window s - 1) against the oracle: identical trajectories, every window
    with flips, fused exchange after each sweep."""
    T = _ladder(0.25, 3.0, 12)
    sim, ref = run_pair(pkg, orc, L, q, 0.45, T, 5 + L, 24, 1, precision=precision, threads=512, steps=2,
                        mode=1)
    assert sim.plan()["threads"] == 512
    obs = _cmp_energy(sim, ref, 1e-6 if precision else 1e-11)
    st = ref.stats()
    np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
    np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])


def test_overlapped_equals_plain_sweep(pkg):
    """The 1024-site workload's shape with and without the overlap: the same
    decisions, energies equal to the rounding of their different summation."""
    T = _ladder(0.3, 3.0, 64)
    out = []
    for threads in (512, 256):
        sim = pkg.Simulation(1024, 3, 0.4, T, 1234, threads=threads)
        sim.run(30, 1)
        out.append((sim.plan()["threads"], sim.spins(), sim.observables()))
        sim.close()
    (t1, (s1, p1), o1), (t2, (s2, p2), o2) = out
    assert (t1, t2) == (512, 256)
    np.testing.assert_array_equal(s1, s2)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_array_equal(o1["flip_acc"], o2["flip_acc"])
    np.testing.assert_allclose(o1["E"], o2["E"], rtol=1e-11)

"""Batched and served runs: every job's trajectory equals the oracle's for the
same job run alone (and the single-instance GPU path), whatever else shares
the launch.  Marked gpu."""
import time

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


def _jobs(n, seed=5, lmax=300, sweeps=(5, 40), rmax=8, qmax=10):
    from workloads import geometric_ladder

    rng = np.random.default_rng(seed)
    out = []
    for j in range(n):
        L = int(rng.integers(2, lmax))
        q = int(rng.integers(2, qmax + 1))
        R = int(rng.integers(1, rmax + 1))
        out.append(dict(L=L, q=q, sigma=float(rng.uniform(0.1, 1.0)), T=geometric_ladder(0.2, 3.0, R),
                        seed=1000 + j, sweeps=int(rng.integers(*sweeps)), exchange_every=int(rng.integers(1, 3)),
                        init=int(rng.integers(0, 2))))
    return out


def _oracle(orc, job):
    ref = orc.PT(job["L"], job["q"], job["sigma"], job["T"], job["seed"], init=job["init"], mode=0, threads=4)
    ref.run(job["sweeps"], job["exchange_every"])
    return ref


def _check_job(orc, job, spins, perm, obs, precision=0):
    """Trajectory exact; energies to 1e-11 relative (FP64 table) or 1e-6 (FP32
    table, whose energy changes are summed from the FP32 couplings)."""
    ref = _oracle(orc, job)
    rs, rp, st = ref.spins(), ref.perm(), ref.stats()
    bad = np.flatnonzero((spins != rs).any(axis=1))
    if bad.size or not np.array_equal(perm, rp):
        print(f"[check] job L={job['L']} q={job['q']} R={len(job['T'])} seed={job['seed']}: walkers with other "
              f"spins {bad.tolist()} ({int((spins != rs).sum())} sites); perm {perm.tolist()} vs {rp.tolist()}; "
              f"flip_acc {obs['flip_acc'].tolist()} vs {st['flip_acc'].tolist()}", flush=True)
    np.testing.assert_array_equal(spins, rs)
    np.testing.assert_array_equal(perm, rp)
    np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
    np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
    rtol = 1e-6 if precision else 1e-11
    np.testing.assert_allclose(obs["E"], ref.energies()[ref.perm()], rtol=rtol, atol=rtol * 100)


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batch_matches_oracle_per_job(pkg, orc, precision):
    jobs = _jobs(24, seed=11 + precision)
    print(f"[batch] {len(jobs)} jobs precision={precision}", flush=True)
    b = pkg.Batch(jobs, precision=precision)
    b.run()
    for j, job in enumerate(jobs):
        s, p = b.spins(j)
        _check_job(orc, job, s, p, b.observables(j), precision)
    b.close()


@pytest.mark.parametrize("threads,lds", [(64, 16384), (128, 65536), (256, 163840), (192, 40000)])
def test_batch_shapes_give_identical_results(pkg, orc, threads, lds):
    """Workgroup size and LDS budget (field table in LDS or in HBM) change no decision."""
    jobs = _jobs(10, seed=3, lmax=700)
    print(f"[batch-shape] threads={threads} lds={lds}", flush=True)
    b = pkg.Batch(jobs, threads=threads, lds_budget=lds)
    b.run()
    for j, job in enumerate(jobs):
        s, p = b.spins(j)
        _check_job(orc, job, s, p, b.observables(j))
    b.close()


def test_batch_equals_single_instance(pkg):
    from workloads import geometric_ladder

    jobs = [dict(L=200, q=3, sigma=0.5, T=geometric_ladder(0.3, 3.0, 12), seed=77, sweeps=30, exchange_every=1, init=0),
            dict(L=64, q=5, sigma=0.3, T=geometric_ladder(0.2, 2.0, 5), seed=78, sweeps=50, exchange_every=2, init=1)]
    b = pkg.Batch(jobs)
    b.run()
    nt = b.shape()["threads"]
    for j, job in enumerate(jobs):
        # same workgroup width: the FP64 energy reductions then run in the same order
        for threads, exact in ((nt, True), (0, False)):
            sim = pkg.Simulation(job["L"], job["q"], job["sigma"], job["T"], job["seed"], init=job["init"],
                                 threads=threads)
            sim.run(job["sweeps"], job["exchange_every"])
            s1, p1 = sim.spins()
            s2, p2 = b.spins(j)
            np.testing.assert_array_equal(s1, s2)
            np.testing.assert_array_equal(p1, p2)
            o1, o2 = sim.observables(), b.observables(j)
            for k in ("flip_acc", "flip_att", "xchg_acc", "sumM2"):
                np.testing.assert_array_equal(o1[k], o2[k])
            if exact:
                np.testing.assert_array_equal(o1["sumE"], o2["sumE"])
            else:
                # another width sums the per-thread FP64 partials in another order
                np.testing.assert_allclose(o1["sumE"], o2["sumE"], rtol=job["L"] ** 2 * 2.0 ** -52)
            sim.close()
    b.close()


def test_batch_job_stats(pkg):
    """Each job's placement as planned and its device start and end clocks:
    start before end, every job inside one launch."""
    from workloads import geometric_ladder

    T = geometric_ladder(0.3, 3.0, 8)
    jobs = [dict(L=64 + 32 * j, q=3, sigma=0.5, T=T, seed=40 + j, sweeps=20 + 30 * j, exchange_every=1, init=0)
            for j in range(6)]
    b = pkg.Batch(jobs)
    with pytest.raises(pkg.PTError):
        b.job_stats(0)  # no clocks before the launch
    b.run()
    st = [b.job_stats(j) for j in range(len(jobs))]
    assert all(s["placement"] == pkg.PLACE_LDS for s in st)
    t0 = np.array([s["start"] for s in st])
    t1 = np.array([s["end"] for s in st])
    assert (t0 < t1).all()
    assert t1.max() - t0.min() < 60.0
    with pytest.raises(pkg.PTError):
        b.job_stats(len(jobs))
    b.close()


def test_batch_more_walkers_than_workgroups(pkg, orc):
    """Far more walkers than resident workgroups: jobs are taken in turn."""
    from workloads import geometric_ladder

    jobs = [dict(L=96, q=3, sigma=0.6, T=geometric_ladder(0.3, 3.0, 32), seed=500 + j, sweeps=6,
                 exchange_every=1, init=0) for j in range(40)]
    b = pkg.Batch(jobs, threads=256, lds_budget=160 * 1024)
    shape = b.shape()
    assert shape["workgroups"] < sum(b.R)
    b.run()
    for j in (0, 17, 39):
        s, p = b.spins(j)
        _check_job(orc, jobs[j], s, p, b.observables(j))
    b.close()


def test_server_results_equal_alone(pkg, orc):
    """Jobs submitted while others run; each equals the oracle run alone."""
    jobs = _jobs(16, seed=21, lmax=400, rmax=16)
    srv = pkg.Server(arena_bytes=64 << 20, max_jobs=64)
    try:  # a server left running keeps every CU: stop it whatever happens
        ids = []
        for k, job in enumerate(jobs):
            ids.append(srv.submit(job))
            if k % 4 == 3:
                time.sleep(0.01)
        for jid, job in zip(ids, jobs):
            obs = srv.wait(jid, timeout=120)
            s, p = srv.spins(jid)
            _check_job(orc, job, s, p, obs)
            t_sub, t_adm, t_fin = srv.times(jid)
            assert t_sub <= t_adm <= t_fin
    finally:
        srv.stop()


def test_server_admission_by_memory(pkg, orc):
    """An arena that holds one job at a time still completes every job."""
    from workloads import geometric_ladder

    jobs = [dict(L=512, q=4, sigma=0.5, T=geometric_ladder(0.3, 3.0, 16), seed=900 + j, sweeps=8,
                 exchange_every=1, init=0) for j in range(4)]
    one = 16 * 512 * 3 * 8 + 16 * 512 + (1 << 16)  # q - 1 stored rows, spins, the rest
    srv = pkg.Server(arena_bytes=one + (one // 2), max_jobs=8)
    try:
        ids = [srv.submit(j) for j in jobs]
        for jid, job in zip(ids, jobs):
            obs = srv.wait(jid, timeout=120)
            s, p = srv.spins(jid)
            _check_job(orc, job, s, p, obs)
        adm = [srv.times(i)[1] for i in ids]
        fin = [srv.times(i)[2] for i in ids]
        for k in range(1, len(ids)):
            assert adm[k] >= fin[k - 1] - 1e-3  # admitted only after the previous job freed its memory
    finally:
        srv.stop()


def test_server_rejects_bad_jobs(pkg):
    srv = pkg.Server(arena_bytes=1 << 20, max_jobs=4)
    try:
        _rejects(pkg, srv)
    finally:
        srv.stop()


def test_server_cancel_queued_jobs(pkg):
    """Jobs beyond the in-flight bound wait on the host and can be cancelled;
    admitted jobs cannot, and every other job still completes."""
    from workloads import geometric_ladder

    T = geometric_ladder(0.3, 3.0, 64)
    jobs = [dict(L=128, q=3, sigma=0.5, T=T, seed=700 + j, sweeps=4000, exchange_every=1, init=0) for j in range(24)]
    srv = pkg.Server(arena_bytes=256 << 20, max_jobs=32)
    try:
        ids = [srv.submit(j) for j in jobs]
        # 1536 walkers: at most twice the resident workgroups are admitted at once
        assert not srv.cancel(ids[0])  # admitted at once (nothing was in flight)
        for jid in ids[-4:]:
            assert srv.cancel(jid)
        assert srv.cancel(ids[-1])  # cancelling twice is harmless
        for jid in ids[:-4]:
            obs = srv.wait(jid, timeout=120)
            assert obs["flip_att"].sum() == 128 * 64 * 4000
        for jid in ids[-4:]:
            with pytest.raises(pkg.PTError):
                srv.poll(jid)
            with pytest.raises(pkg.PTError):
                srv.wait(jid, timeout=1)
            with pytest.raises(pkg.PTError):
                srv.spins(jid)
        assert not srv.cancel(ids[1])  # finished
    finally:
        srv.stop()


def _rejects(pkg, srv):
    with pytest.raises(pkg.PTError):
        srv.submit(dict(L=10, q=3, sigma=0.0, T=[1.0], seed=1, sweeps=1))
    with pytest.raises(pkg.PTError):
        srv.submit(dict(L=10, q=3, sigma=0.5, T=np.linspace(0.5, 2.0, 65), seed=1, sweeps=1))


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_batch_with_largest_job_shapes(pkg, orc, precision):
    """Jobs at the extremes of the 256-job batched workload (L up to 8192, q up
    to 10, 32 replicas geometric in [0.2, 3.0]) in one launch at the default
    shape, each against the oracle on all its walkers."""
    import workloads
    from workloads import geometric_ladder

    T = geometric_ladder(0.2, 3.0, 32)
    jobs = [dict(L=8192, q=10, sigma=0.55, T=T, seed=1234, sweeps=3, exchange_every=1, init=0),
            dict(L=1000, q=3, sigma=0.4, T=T, seed=1235, sweeps=20, exchange_every=1, init=0),
            dict(L=128, q=2, sigma=1.0, T=T, seed=1236, sweeps=40, exchange_every=1, init=0)]
    for j in workloads.batch_jobs(n_jobs=3, sweeps=4):
        jobs.append(dict(L=j.L, q=j.q, sigma=j.sigma, T=j.T, seed=j.seed, sweeps=j.sweeps, exchange_every=1, init=0))
    print(f"[batch-large] {[(j['L'], j['q']) for j in jobs]} precision={precision}", flush=True)
    b = pkg.Batch(jobs, precision=precision)
    b.run()
    for j, job in enumerate(jobs):
        s, p = b.spins(j)
        obs = b.observables(j)
        ref = orc.PT(job["L"], job["q"], job["sigma"], job["T"], job["seed"], init=job["init"], mode=0, threads=16)
        ref.run(job["sweeps"], job["exchange_every"])
        np.testing.assert_array_equal(s, ref.spins())
        np.testing.assert_array_equal(p, ref.perm())
        st = ref.stats()
        np.testing.assert_array_equal(obs["flip_acc"], st["flip_acc"])
        np.testing.assert_array_equal(obs["xchg_acc"], st["xchg_acc"])
        rtol = max(1e-11, job["L"] ** 2 / 2 * 2.0**-53) if not precision else 1e-6
        np.testing.assert_allclose(obs["E"], ref.energies()[ref.perm()], rtol=rtol)
    b.close()

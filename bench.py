"""Benchmark: spin-flip attempts per second of parallel tempering for the 1D
long-range q-state Potts ring on one MI355X.

One step = the whole hot path on one batch of synthetic input: couplings J*
from the Hurwitz-zeta kernel, initial spins, the O(L^2) field table, then the
sweeps (L Metropolis attempts per replica each) with a two-stage exchange step
after every sweep, and the observables.  The default workload is L = 1024,
q = 3, sigma = 0.4, 64 replicas with temperatures geometric in [0.3, 3.0],
uniform random spins from seed 1234, 10^4 sweeps.

Prints one JSON line (rank 0).  `value` is attempts/s = L * R * sweeps * steps
/ time, timed between two synchronisations with the state's workspace already
allocated in HBM.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks and unit counts
CUS = 256
CLOCK_HZ = 2.4e9
# LDS read bandwidth per CU per clock.  CDNA 3 reads 128 B/clk from its 64 KB
# LDS; CDNA 4 (gfx950) grows the LDS to 160 KB and doubles its read bandwidth
# (AMD CDNA 4 architecture whitepaper), so 256 B/clk/CU: 157.3 TB/s for the
# chip.  The probe (conflict-free 16-byte reads) reaches about 107 TB/s, more
# than a 128 B/clk model allows, so that model cannot be the ceiling.
LDS_BYTES_PER_CLK_CU = 256
LDS_PEAK = CUS * LDS_BYTES_PER_CLK_CU * CLOCK_HZ  # 157.3 TB/s
HBM_PEAK = 8.0e12
PLACE_NAMES = {1: "lds", 2: "hbm", 3: "direct"}
PRECS = {"f64": 0, "f32": 1, "i32": 2}
PREC_NAMES = {0: "f64", 1: "f32", 2: "i32"}
TABLE_NAMES = {0: "fp64", 1: "fp32 + fp64 recheck", 2: "int32 fixed point + fp64 recheck"}


def workload(name):
    import workloads

    return {"small": workloads.small, "medium": workloads.medium, "large": workloads.large}[name]()


def kernel_source_sha():
    """Hash of the sources libptmi.so is built from (the probe library's own
    source excluded), so a committed counter summary stays tied to the kernel
    it measured."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_1308_5426_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f == "lds_probe.hip":
            continue
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(obs, inst, prec, placement):
    """Bytes the method must move per launch, by placement of the field table.

    Table in HBM (f bytes per entry; the bound is HBM): per attempt two table
    entries (2 f), per accepted flip two table rows read and written (4 f L), per
    refresh the table written (f q L).
    Table in LDS (f = 4 B FP32 / int32, 8 B FP64 per entry): per attempt the spin s_i
    and two table entries (1 + 2 f); per accepted flip one coupling row read
    and two table rows read and written (5 f L); per refresh one FP64 coupling
    per site pair (8 L^2); per recheck one FP64 coupling and one spin per site
    (9 L).  No table (direct sums): per attempt one spin and one FP64 coupling
    per site (9 L).  Both: per walker and sweep the energy and magnetisation
    reductions read 5 L; per exchange step 8 R of energies."""
    fb = 8 if prec == 0 else 4
    acc = int(obs["flip_acc"].sum())
    attempts = inst.L * inst.R * inst.sweeps
    common = inst.R * inst.sweeps * 5 * inst.L + obs["exchange_steps"] * 8 * inst.R
    if placement == 3:
        return attempts * 9 * inst.L + common, acc
    if placement == 2:  # the table's side in HBM: two entries per attempt, two rows read and written per flip
        return attempts * 2 * fb + acc * 4 * fb * inst.L + obs["n_refresh"] * fb * inst.q * inst.L, acc
    return (attempts * (1 + 2 * fb) + acc * 5 * fb * inst.L + obs["n_refresh"] * 8 * inst.L * inst.L
            + obs["n_recheck"] * 9 * inst.L + common), acc


def phase_summary(ph, inst, prec, placement):
    """Phase counters of a profiled run: where each walker's cycles went, and
    the field update measured where it runs (flush cycles inside the sweep
    kernel) against the LDS peak of one CU."""
    import numpy as np

    fb = 8 if prec == 0 else 4
    tot = ph["total"].astype(float)
    share = {k: float(ph[k].sum() / tot.sum()) for k in ("draw", "chain", "flush", "record", "exchange")}
    hot = int(np.argmax(ph["flips"]))
    out = {"cycles_share": share,
           "iters_per_window": float(ph["iters"].sum() / max(1, ph["windows"].sum())),
           "flips_per_flushed_window": float(ph["flips"].sum() / max(1, ph["flushes"].sum())),
           "hottest_walker": {"walker": hot, "flips": int(ph["flips"][hot]),
                              "cycles_share": {k: float(ph[k][hot] / tot[hot])
                                               for k in ("draw", "chain", "flush", "record", "exchange")},
                              "iters_per_window": float(ph["iters"][hot] / max(1, ph["windows"][hot])),
                              # the chain's cycles by step of its guess-and-check iterations
                              "chain_split": {k[6:]: float(ph[k][hot] / max(1, ph["chain"][hot]))
                                              for k in ("chain_guess", "chain_correct", "chain_check",
                                                        "chain_resolve", "chain_redo", "chain_sync")}}}
    if placement != 3 and ph["flush"].sum() > 0:
        # algorithmic field-update bytes (5 f L per flip) per flush cycle of each
        # walker's workgroup, i.e. per CU, against 256 B/clk/CU
        b = ph["flips"].astype(float) * 5 * fb * inst.L
        per_clk = b.sum() / ph["flush"].sum()
        out["field_update_in_sweep"] = {
            "bytes_per_clk_per_cu": per_clk, "peak_bytes_per_clk_per_cu": LDS_BYTES_PER_CLK_CU,
            "frac": per_clk / LDS_BYTES_PER_CLK_CU,
            "hottest_walker_frac": float(b[hot] / ph["flush"][hot] / LDS_BYTES_PER_CLK_CU),
            "note": "flush cycles inside k_sweep (s_memtime by thread 0 between the barriers around each "
                    "window's flush); 5 f L algorithmic bytes per accepted flip"}
    return out


def run_gpu(inst, prec, steps, warmup, max_chunk=0, placement=0, threads=0):
    import torch

    import paper_1308_5426_amd as pkg

    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t_kernel = []
    obs_last = None
    plan = None

    def one_step(timed, profile=False):
        nonlocal obs_last, plan
        sim = pkg.Simulation(inst.L, inst.q, inst.sigma, inst.T, inst.seed, precision=prec, init=inst.init,
                             max_sweeps_per_launch=max_chunk or inst.sweeps, placement=placement, profile=profile,
                             threads=threads)
        plan = sim.plan()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        print(f"[bench] instance ready ({PLACE_NAMES.get(plan['placement'])}, {plan['threads']} threads, "
              f"{plan['lds_bytes']} B LDS{', profiled' if profile else ''}), running {inst.sweeps} sweeps",
              file=sys.stderr, flush=True)
        e0.record(stream)
        done = 0
        while done < inst.sweeps:  # long runs go in launches of max_chunk sweeps, each reported
            n = min(inst.sweeps - done, max_chunk or inst.sweeps)
            sim.run(n, 1)
            done += n
            if done < inst.sweeps:
                sim.synchronize()
                print(f"[bench] {done} sweeps", file=sys.stderr, flush=True)
        e1.record(stream)
        obs = sim.observables()  # synchronises
        print(f"[bench] sweeps done in {e0.elapsed_time(e1) / 1e3:.2f} s", file=sys.stderr, flush=True)
        if timed:
            t_kernel.append(e0.elapsed_time(e1) / 1e3)
            obs_last = obs
        ph = sim.phase_counters() if profile else None
        # the workspace returns to PyTorch's cache and is reused by the next step
        sim.close()
        return ph

    for _ in range(warmup):
        one_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return elapsed, t_kernel, obs_last, plan, one_step


def _oracle_rate(inst, seconds, mode, threads):
    """Attempts/s of the oracle on `threads` host threads over about `seconds`
    of sweeps 2.. of the workload (sweep 1 sizes the sample)."""
    import oracle

    pt = oracle.PT(inst.L, inst.q, inst.sigma, inst.T, inst.seed, init=inst.init, mode=mode, threads=threads)
    t0 = time.perf_counter()
    pt.run(1, 1)
    t1 = time.perf_counter() - t0
    n = max(1, int(seconds / max(t1, 1e-6)))
    t0 = time.perf_counter()
    pt.run(n, 1)
    dt = time.perf_counter() - t0
    pt.close()
    return inst.L * inst.R * n / dt, n, dt


def field_update_alone(inst, peak, flips=65536, reps=4):
    """The sweep kernel's flush replayed alone (one workgroup per replica,
    accept-like flips at the workload's L and q) against the same LDS peak."""
    import workloads
    from paper_1308_5426_amd import flush_bench

    words, _ = workloads.flip_sequence(inst.L, inst.q, flips, inst.seed)
    J = flush_bench.jstar(inst.L, inst.sigma)
    _, ms = flush_bench.replay(J, inst.q, words, inst.R, reps)
    achieved = 40.0 * inst.L * flips * reps * inst.R / (ms * 1e-3)
    return {"kernel": "k_flush_replay (flush_window alone)", "workgroups": inst.R, "flips": flips * reps * inst.R,
            "ms": ms, "achieved": achieved / 1e9, "unit": "GB/s", "peak": peak / 1e9, "frac": achieved / peak,
            "frac_occupied_cus": achieved / (peak * min(inst.R, CUS) / CUS)}


def cpu_baseline(inst, seconds=12.0, mode=0):
    """The oracle on this host's cores, on the first sweeps of the same workload:
    the direct O(L) mode on all cores (the reported value), and shorter samples
    of the same mode on one core and of the FP64 field-table mode on all cores."""
    threads = min(16, os.cpu_count() or 1)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    rate, n, dt = _oracle_rate(inst, seconds, mode, threads)
    one, n1, dt1 = _oracle_rate(inst, seconds / 4, mode, 1)
    tab, n2, dt2 = _oracle_rate(inst, seconds / 4, 1 - mode, threads)
    what = "direct O(L) energy difference" if mode == 0 else "FP64 field table"
    other = "FP64 field table" if mode == 0 else "direct O(L) energy difference"
    return {"value": rate, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "nproc": os.cpu_count(), "cpu_model": model,
            "sample": f"sweeps 2..{n + 1} of the same workload ({inst.R} replicas x {inst.L} sites, exchange "
                      f"after each sweep), oracle mode: {what}, {dt:.1f} s; also {n1} sweeps on 1 core "
                      f"({dt1:.1f} s) and {n2} sweeps of the {other} mode on {threads} threads ({dt2:.1f} s)",
            "value_1core": one, "value_other_mode": tab}


def run_batch(args):
    """256 uneven jobs in one persistent launch vs the plain per-instance form."""
    import torch

    import paper_1308_5426_amd as pkg
    import workloads
    from paper_1308_5426_amd import autotune

    jobs = workloads.batch_jobs(n_jobs=args.jobs, sweeps=args.sweeps or 1000)
    prec = PRECS[args.precision]
    jd = [dict(L=j.L, q=j.q, sigma=j.sigma, T=j.T, seed=j.seed, sweeps=j.sweeps, exchange_every=1, init=0)
          for j in jobs]
    threads, lds = (autotune.tune(jd, precision=prec, verbose=True) if args.autotune else (args.threads, args.lds))
    attempts = sum(j.L * j.R * j.sweeps for j in jobs)
    times, shape = [], None
    for it in range(args.warmup + args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = pkg.Batch(jd, precision=prec, threads=threads, lds_budget=lds)
        b.run()
        acc = sum(int(b.observables(j)["flip_acc"].sum()) for j in range(len(jd)))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        shape = b.shape()
        stats = [b.job_stats(j) for j in range(len(jd))]
        b.close()
        if it >= args.warmup:
            times.append(dt)
        print(f"[batch] step {it} ({'timed' if it >= args.warmup else 'warm-up'}) {dt:.2f} s", file=sys.stderr,
              flush=True)
    el = sum(times)
    breakdown = batch_breakdown(jd, stats, shape["workgroups"])
    # plain per-instance GPU form: the same jobs one pt_init/pt_run at a time
    k = min(args.plain_sample, len(jd))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for n_done, j in enumerate(jd[:k]):
        sim = pkg.Simulation(j["L"], j["q"], j["sigma"], j["T"], j["seed"], precision=prec)
        sim.run(j["sweeps"], 1)
        sim.observables()
        sim.close()
        print(f"[batch] plain job {n_done} done", file=sys.stderr, flush=True)
    dt_plain = time.perf_counter() - t0
    att_plain = sum(j["L"] * len(j["T"]) * j["sweeps"] for j in jd[:k])
    return {
        "metric": "spin-flip attempts/sec (all replicas, batched)",
        "value": attempts * args.steps / el, "unit": "attempts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": PREC_NAMES[prec], "data": "synthetic",
        "config": {"workload": f"{len(jd)} jobs, L log-uniform [128, 8192], q in 2..10, sigma in [0.1, 1], "
                               f"32 replicas geometric [0.2, 3.0], {jd[0]['sweeps']} sweeps, exchange every sweep",
                   "jobs": len(jd), "walkers": sum(len(j["T"]) for j in jd), "attempts": attempts,
                   "accept_fraction": acc / attempts, "shape": shape, "autotuned": bool(args.autotune)},
        "plain_per_instance": {"value": att_plain / dt_plain, "unit": "attempts/s", "jobs_timed": k,
                               "seconds": dt_plain},
        "breakdown": breakdown,
    }


def batch_breakdown(jd, stats, workgroups):
    """Where a batched launch's time went, from each job's device start and
    end clocks: the launch span, the fraction of walker slots busy over it,
    the time spent with fewer than half the slots busy, and each placement's
    share of jobs, attempts and walker-seconds."""
    import numpy as np

    t0 = np.array([st["start"] for st in stats])
    t1 = np.array([st["end"] for st in stats])
    R = np.array([len(j["T"]) for j in jd], float)
    att = np.array([j["L"] * len(j["T"]) * j["sweeps"] for j in jd], float)
    span = float(t1.max() - t0.min())
    ws = R * (t1 - t0)
    grid = np.linspace(t0.min(), t1.max(), 2001)
    busy = np.array([R[(t0 <= t) & (t < t1)].sum() for t in grid]) / workgroups
    names = {1: "lds", 2: "hbm", 3: "direct"}
    by = {}
    for p, name in names.items():
        m = np.array([st["placement"] == p for st in stats])
        if m.any():
            by[name] = {"jobs": int(m.sum()), "attempts_share": float(att[m].sum() / att.sum()),
                        "walker_seconds_share": float(ws[m].sum() / ws.sum()),
                        "attempts_per_walker_second": float(att[m].sum() / ws[m].sum())}
    return {"device_span_s": span, "busy_fraction": float(ws.sum() / (workgroups * span)),
            "seconds_below_half_busy": float((busy < 0.5).mean() * span),
            "last_job_start_to_end_s": float(t1.max() - t0.max()), "by_placement": by}


def run_serve(args):
    """Poisson arrivals; each job submitted at its arrival time; time to result."""
    import numpy as np
    import torch

    import paper_1308_5426_amd as pkg
    import workloads

    stream = workloads.serve_stream(rate=args.rate, duration=args.duration)
    prec = PRECS[args.precision]
    # synchronise before the server starts: a device-wide synchronisation would
    # wait for the server's resident kernel, which runs until stop()
    torch.cuda.synchronize()
    srv = pkg.Server(arena_bytes=int(args.arena_gb * (1 << 30)), max_jobs=len(stream) + 16, precision=prec,
                     threads=args.threads, lds_budget=args.lds)
    print(f"[serve] server up, {len(stream)} jobs to submit", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ids = []
    for (ta, inst) in stream:
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        ids.append((ta, inst, srv.submit(dict(L=inst.L, q=inst.q, sigma=inst.sigma, T=inst.T, seed=inst.seed,
                                              sweeps=inst.sweeps, exchange_every=1, init=0))))
        if len(ids) % 200 == 0:
            print(f"[serve] submitted {len(ids)} at t={time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    lat, cens, done_t, att, dropped = [], [], [], 0, set()
    horizon = args.horizon if args.horizon > 0 else None
    cut = False
    for n_done, (ta, inst, jid) in enumerate(ids):
        if not cut:
            left = 600.0 if horizon is None else max(0.01, horizon - (time.perf_counter() - t0))
            try:
                srv.wait(jid, timeout=left)
            except pkg.PTError:
                if horizon is None or time.perf_counter() - t0 < horizon:
                    raise
                # horizon reached: drop what still waits on the host; admitted jobs run to their end
                cut = True
                dropped = {j for (_, _, j) in ids[n_done:] if srv.cancel(j)}
                print(f"[serve] horizon {horizon:g} s: {len(dropped)} queued jobs cancelled", file=sys.stderr, flush=True)
        if cut and jid in dropped:
            sub, _, fin = srv.times(jid)
            lat.append(fin - sub)
            cens.append(True)
            continue
        srv.wait(jid, timeout=600)
        if n_done % 100 == 99:
            print(f"[serve] {n_done + 1} results", file=sys.stderr, flush=True)
        sub, adm, fin = srv.times(jid)
        lat.append(fin - sub)
        cens.append(False)
        done_t.append(fin)
        att += inst.L * inst.R * inst.sweeps
    span = max(done_t) - min(srv.times(j)[0] for (_, _, j) in ids)
    srv.stop()
    lat, cens = np.array(lat), np.array(cens)

    def pct(qv):
        # nearest-rank percentile over all jobs; a cancelled job's time to
        # result is at least its wait until cancellation, so the figure is a
        # lower bound unless every cancelled job's wait already exceeds it
        order = np.argsort(lat, kind="stable")
        k = max(0, int(np.ceil(qv / 100.0 * len(lat))) - 1)
        v = float(lat[order[k]])
        exact = not cens[order[: k + 1]].any()
        return v, exact

    p50, p50x = pct(50)
    p99, p99x = pct(99)
    done_lat = lat[~cens]
    return {
        "metric": "spin-flip attempts/sec (all replicas, served); p50/p99 time-to-result",
        "value": att / span, "unit": "attempts/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": span * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": PREC_NAMES[prec], "data": "synthetic",
        "config": {"workload": f"Poisson {args.rate:g} jobs/s for {args.duration:g} s; L log-uniform [64, 4096], "
                               "q in 2..8, sigma in [0.1, 1], 16-64 replicas, 500-5000 sweeps",
                   "jobs": len(ids), "attempts": att},
        "latency_s": {"p50": p50, "p50_exact": p50x, "p99": p99, "p99_exact": p99x,
                      "completed_p50": float(np.percentile(done_lat, 50)),
                      "completed_p99": float(np.percentile(done_lat, 99)),
                      "completed_max": float(done_lat.max())},
        "jobs_completed": int((~cens).sum()), "jobs_cancelled": int(cens.sum()),
        "horizon_s": horizon,
    }


def lds_peak_measured():
    """Aggregate LDS read bandwidth of the device from the probe library
    (conflict-free 16-byte reads, 2 workgroups of 1024 threads per CU)."""
    import ctypes

    path = os.path.join(ROOT, "paper_1308_5426_amd", "libptmi_probe.so")
    lib = ctypes.CDLL(path)
    lib.ptmi_lds_read_bandwidth.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_double)]
    bw = ctypes.c_double(0.0)
    if lib.ptmi_lds_read_bandwidth(2 * CUS, 1024, 2000, ctypes.byref(bw)) != 0:
        return None
    return bw.value


def load_traffic(sha, key):
    """Counter figures of the sweep kernel from the committed summaries in
    profiles/ (lines `key: value`) whose workload key and kernel-source hash
    match: LDS bytes per launch (SQ_INSTS_LDS_*_BANDWIDTH x 64 B) and HBM bytes
    per launch (FETCH_SIZE and WRITE_SIZE, calibrated by a copy kernel)."""
    out = {}
    d = os.path.join(ROOT, "profiles")
    for name in sorted(os.listdir(d)):
        vals = {}
        with open(os.path.join(d, name)) as f:
            for line in f:
                if ":" in line and not line.startswith(("#", "`", " ", "|")):
                    k, v = line.split(":", 1)
                    vals[k.strip()] = v.strip()
        if vals.get("key") != key or vals.get("source_sha") != sha:
            continue
        for k in ("lds_bytes_per_launch", "hbm_bytes_per_launch"):
            if k in vals:
                out[k] = float(vals[k])
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="medium", choices=["small", "medium", "large", "batch", "serve"])
    ap.add_argument("--jobs", type=int, default=256, help="batch: number of jobs")
    ap.add_argument("--plain-sample", type=int, default=8, help="batch: jobs timed one at a time")
    ap.add_argument("--autotune", action="store_true", help="batch: measure the workgroup shape first")
    ap.add_argument("--rate", type=float, default=50.0, help="serve: arrivals per second")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--arena-gb", type=float, default=16.0, help="serve: device arena")
    ap.add_argument("--horizon", type=float, default=0.0,
                    help="serve: seconds after the first arrival at which jobs still queued are cancelled (0: none)")
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--precision", default="f64", choices=list(PRECS))
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first copy this many bytes device to device (a kernel of known HBM traffic, "
                         "to calibrate the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--sweeps", type=int, default=0, help="override the workload's sweep count")
    ap.add_argument("--placement", default="auto", choices=["auto", "lds", "hbm", "direct"],
                    help="field table placement of single instances")
    ap.add_argument("--no-profile", action="store_true", help="skip the profiled pass (phase counters)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload of the default run")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(walkers would shard across GPUs with an all-gather of R energies per exchange step)",
              file=sys.stderr)
        sys.exit(2)

    if args.workload in ("batch", "serve"):
        out = run_batch(args) if args.workload == "batch" else run_serve(args)
        print(json.dumps(out), flush=True)
        return

    if args.copy_bytes:
        import torch

        src = torch.ones(args.copy_bytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    inst = workload(args.workload)
    if args.sweeps:
        inst.sweeps = args.sweeps
    prec = PRECS[args.precision]
    placement = {"auto": 0, "lds": 1, "hbm": 2, "direct": 3}[args.placement]
    # the L = 16384 instance runs in launches of 250 sweeps (progress between them)
    elapsed, tk, obs, plan, one_step = run_gpu(inst, prec, args.steps, args.warmup,
                                               max_chunk=250 if inst.L > 8192 else 0, placement=placement,
                                               threads=args.threads)
    attempts = inst.L * inst.R * inst.sweeps
    value = attempts * args.steps / elapsed
    kern = sum(tk) / len(tk)
    bytes_, acc = algorithmic_bytes(obs, inst, prec, plan["placement"])
    achieved = bytes_ / kern
    sha = kernel_source_sha()
    tr = load_traffic(sha, f"{args.workload}_{args.precision}_{PLACE_NAMES[plan['placement']]}")
    occupied = min(CUS, inst.R)
    lds_meas = lds_peak_measured()
    hbm_bound = plan["placement"] == 2
    peak = HBM_PEAK if hbm_bound else LDS_PEAK
    out = {
        "metric": "spin-flip attempts/sec (all replicas)",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_NAMES[prec],
        "data": "synthetic",
        "config": {
            "workload": f"L={inst.L} q={inst.q} sigma={inst.sigma} R={inst.R} T geometric "
                        f"[{inst.T[0]:g},{inst.T[-1]:g}] sweeps={inst.sweeps} exchange every sweep "
                        f"{'ordered' if inst.init else 'uniform random'} spins seed={inst.seed}",
            "L": inst.L, "q": inst.q, "sigma": inst.sigma, "replicas": inst.R, "sweeps": inst.sweeps,
            "field_table": TABLE_NAMES[prec] + " in " + PLACE_NAMES[plan["placement"]],
            "threads_per_walker": plan["threads"], "lds_bytes_per_walker": plan["lds_bytes"],
        },
        "roofline": {
            "bound": "hbm" if hbm_bound else "lds",
            "kernel": "k_sweep (persistent, exchange fused)",
            "achieved": achieved / 1e9,
            "peak": peak / 1e9,
            "unit": "GB/s",
            "frac": achieved / peak,
            "frac_occupied_cus": achieved / (peak * occupied / CUS),
            "peak_note": "8 TB/s HBM3E" if hbm_bound else
                         "256 B/clk/CU x 256 CUs x 2.4 GHz (CDNA 4 LDS read bandwidth); the probe's measured "
                         "rate is an achievable reference, not the peak",
            "probe_measured": None if lds_meas is None else lds_meas / 1e9,
            "traffic": tr.get("lds_bytes_per_launch"),
            "traffic_note": "LDS bytes per launch measured by SQ_INSTS_LDS_LOAD/STORE/ATOMIC_BANDWIDTH (64 B units, "
                            "exact on the LDS probe) in the committed counter summary of these kernel sources, "
                            "else null",
            "hbm_traffic": tr.get("hbm_bytes_per_launch"),
            "hbm_traffic_note": "HBM bytes per launch: FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for "
                                "a 1 GiB device copy, from the committed summary of these kernel sources, else null",
            "kernel_ms": kern * 1e3,
            "algorithmic_bytes_per_launch": bytes_,
            "accepted_flips_per_launch": acc,
            "acceptance": acc / attempts,
            "rechecks_per_launch": obs["n_recheck"],
            "refreshes_per_launch": obs["n_refresh"],
            "exact_energies_per_launch": obs["n_exact_energy"],
            "source_sha": sha,
        },
    }
    if not args.no_profile:
        # one more (untimed) pass of the same step with the phase counters on
        print("[bench] profiled pass", file=sys.stderr, flush=True)
        ph = one_step(False, profile=True)
        out["phases"] = phase_summary(ph, inst, prec, plan["placement"])
    if not prec and inst.q <= 4 and inst.L <= 3000:
        out["field_update_alone"] = field_update_alone(inst, LDS_PEAK)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_seconds, mode=0)
    if args.workload == "medium" and not args.no_batch:
        print("[bench] batched workload: 256 jobs x 1000 sweeps in one launch", file=sys.stderr, flush=True)
        b = run_batch(argparse.Namespace(jobs=256, sweeps=1000, precision=args.precision, autotune=False,
                                         threads=0, lds=0, steps=1, warmup=0, plain_sample=args.plain_sample))
        out["batched"] = {"metric": b["metric"], "value": b["value"], "unit": b["unit"],
                          "seconds": b["ms_per_step"] / 1e3, "config": b["config"],
                          "plain_per_instance": b["plain_per_instance"],
                          "batched_over_plain": b["value"] / b["plain_per_instance"]["value"],
                          "breakdown": b["breakdown"]}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

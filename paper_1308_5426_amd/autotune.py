"""Measured choice of the walker workgroup shape for batches and servers.

Two knobs decide how a batch maps onto the chip: threads per walker
workgroup (64..256; more threads speed up the O(L) flush and the O(L^2)
table build of one walker, fewer let more walkers share a CU) and the LDS
budget per workgroup (a larger budget keeps more field tables in LDS instead
of HBM but leaves room for fewer workgroups per CU).  The tuner runs a
shortened copy of the batch (same jobs, fewer sweeps) for each candidate,
keeps the fastest in attempts per second, and caches the choice in a JSON
file keyed by the batch's shape signature (environment variable
PT_AUTOTUNE_CACHE, default ~/.cache/ptmi_autotune.json).
"""
from __future__ import annotations

import json
import math
import os
import time

THREADS = (64, 128, 256)
LDS_BUDGETS = (24 * 1024, 48 * 1024, 80 * 1024, 160 * 1024)


def cache_path() -> str:
    return os.environ.get("PT_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "ptmi_autotune.json"))


def _get(job, k, d=None):
    return job.get(k, d) if isinstance(job, dict) else getattr(job, k, d)


def signature(jobs, precision) -> str:
    """Coarse description of a batch: precision, job count, and the walker
    count in each (log2 L, q <= 4) bucket."""
    buckets = {}
    for j in jobs:
        key = (int(math.log2(max(2, _get(j, "L")))), int(_get(j, "q") <= 4))
        buckets[key] = buckets.get(key, 0) + len(_get(j, "T"))
    items = ",".join(f"{a}:{b}:{n}" for (a, b), n in sorted(buckets.items()))
    return f"p{precision}|n{len(jobs)}|{items}"


def _load():
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass


def _shorten(job, frac, min_sweeps):
    j = dict(job) if isinstance(job, dict) else {k: _get(job, k) for k in
                                                 ("L", "q", "sigma", "T", "seed", "sweeps", "init")}
    j.setdefault("exchange_every", _get(job, "exchange_every", 1) or 1)
    j["sweeps"] = max(min_sweeps, int(round(_get(job, "sweeps") * frac)))
    return j


def tune(jobs, precision=0, frac=0.05, min_sweeps=5, candidates=None, use_cache=True, verbose=False):
    """Return (threads, lds_budget) for this batch, measuring if not cached."""
    import torch

    import paper_1308_5426_amd as pkg

    sig = signature(jobs, precision)
    cache = _load() if use_cache else {}
    if sig in cache:
        c = cache[sig]
        return int(c["threads"]), int(c["lds_budget"])
    probe = [_shorten(j, frac, min_sweeps) for j in jobs]
    attempts = sum(j["L"] * len(j["T"]) * j["sweeps"] for j in probe)
    best, results = None, []
    for threads in (candidates or [(t, b) for t in THREADS for b in LDS_BUDGETS]):
        t, b = threads if isinstance(threads, tuple) else threads
        try:
            batch = pkg.Batch(probe, precision=precision, threads=t, lds_budget=b)
        except pkg.PTError:
            continue  # e.g. too few resident workgroups for the largest job
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batch.run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        batch.close()
        rate = attempts / dt
        results.append((t, b, rate))
        if verbose:
            print(f"[autotune] threads={t} lds={b} {rate:.3e} attempts/s", flush=True)
        if best is None or rate > best[2]:
            best = (t, b, rate)
    if best is None:
        raise RuntimeError("no workgroup shape can run this batch")
    cache[sig] = {"threads": best[0], "lds_budget": best[1], "rate": best[2],
                  "tried": [list(r) for r in results]}
    if use_cache:
        _store(cache)
    return best[0], best[1]

"""The field update alone against the LDS roofline.

Replays a sequence of accepted flips, 64 per window, through the sweep
kernel's flush (the O(L) update h[old][.] -= J*(. - i), h[new][.] += J*(. - i)
per accepted flip) on an FP64 table in LDS, one copy per workgroup, and
reports its algorithmic LDS bytes (8 L of couplings read, two rows of 8 L read
and written: 40 L B per flip) per second against the measured LDS read peak of
the device.  The sequence has the statistics of accepted flips in a sweep:
uniform sites, the old state the site's current one, the new state uniform
over the others, starting from all spins in state 0.

    python -m paper_1308_5426_amd.flush_bench --L 1024 --q 3 --flips 65536
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

import numpy as np

from . import LIB_PATH, Simulation

PROBE_PATH = os.path.join(os.path.dirname(LIB_PATH), "libptmi_probe.so")
_probe = None


def probe():
    """The probe library (raises if it has not been built; no CPU fallback)."""
    global _probe
    if _probe is None:
        if not os.path.exists(PROBE_PATH):
            raise ImportError(f"{PROBE_PATH} is missing: build it with __graft_entry__.build()")
        import torch  # noqa: F401  (its HIP runtime first, as for the main library)

        lib = ctypes.CDLL(PROBE_PATH)
        P = ctypes.c_void_p
        lib.ptmi_flush_replay.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_int32, P, ctypes.POINTER(ctypes.c_double)]
        lib.ptmi_flush_replay.restype = ctypes.c_int
        lib.ptmi_lds_read_bandwidth.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_double)]
        lib.ptmi_lds_read_bandwidth.restype = ctypes.c_int
        lib.ptmi_valu_issue_rate.argtypes = [ctypes.c_int32] * 4 + [ctypes.POINTER(ctypes.c_double)] * 2
        lib.ptmi_valu_issue_rate.restype = ctypes.c_int
        _probe = lib
    return _probe


def fields(J, s, q):
    """h[k][j] = sum_{i != j} J*(|i - j| mod L) [s_i = k] (J*(0) = 0), FP64."""
    L = len(s)
    d = (np.arange(L)[None, :] - np.arange(L)[:, None]) % L
    Jm = J[d]
    return np.stack([(Jm * (s == k)[:, None]).sum(axis=0) for k in range(q)])


def jstar(L, sigma):
    """J*(r) from the library's own GPU kernel."""
    with Simulation(L, 2, sigma, [1.0], 1) as sim:
        return sim.jstar()


def replay(J, q, words, workgroups, reps):
    L = len(J)
    h0 = np.zeros((q, L))
    h0[0, :] = J[1:].sum()  # all spins in state 0
    out = np.zeros((q, L))
    ms = ctypes.c_double(0.0)
    w = np.ascontiguousarray(words, np.uint32)
    rc = probe().ptmi_flush_replay(L, q, J.ctypes.data, h0.ctypes.data, w.ctypes.data, len(w), workgroups, reps,
                                   out.ctypes.data, ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError(f"ptmi_flush_replay failed ({rc})")
    return out, ms.value


def lds_peak():
    bw = ctypes.c_double(0.0)
    rc = probe().ptmi_lds_read_bandwidth(512, 1024, 2000, ctypes.byref(bw))  # as bench.py measures it
    if rc != 0:
        raise RuntimeError(f"ptmi_lds_read_bandwidth failed ({rc})")
    return bw.value


VALU_KINDS = ("fp64_fma", "fp32_fma")


def valu_issue(kind, threads, iters=20000, blocks=256):
    """Time between two issues of one VALU instruction kind by one wave, in ns,
    with threads/64 waves per CU (one workgroup per CU: `blocks` = the CU
    count), and the checksum the probe returns (120 + 16 iters)."""
    ms, s = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = probe().ptmi_valu_issue_rate(VALU_KINDS.index(kind), blocks, threads, iters, ctypes.byref(ms), ctypes.byref(s))
    if rc != 0:
        raise RuntimeError(f"ptmi_valu_issue_rate failed ({rc})")
    waves_per_simd = max(1, threads // 256)
    return ms.value * 1e6 / (16.0 * iters * waves_per_simd), s.value


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--L", type=int, default=1024)
    ap.add_argument("--q", type=int, default=3)
    ap.add_argument("--sigma", type=float, default=0.4)
    ap.add_argument("--flips", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=4)
    ap.add_argument("--workgroups", default="64,256")
    ap.add_argument("--seed", type=int, default=1234)
    a = ap.parse_args(argv)
    import sys

    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads  # the seeded input generators (repository root)

    J = jstar(a.L, a.sigma)
    words, s = workloads.flip_sequence(a.L, a.q, a.flips, a.seed)
    h1, _ = replay(J, a.q, words, 1, 1)
    err = float(np.max(np.abs(h1 - fields(J, s, a.q))))
    peak = lds_peak()
    runs = []
    for wg in (int(x) for x in a.workgroups.split(",")):
        _, ms = replay(J, a.q, words, wg, a.reps)
        flips = a.flips * a.reps * wg
        rate = 40.0 * a.L * flips / (ms * 1e-3)
        runs.append({"workgroups": wg, "ms": round(ms, 3), "flips_per_s": flips / (ms * 1e-3),
                     "lds_GBps": rate / 1e9, "frac_of_peak": rate / peak,
                     "frac_of_occupied_cus": rate / (peak * min(wg, 256) / 256)})
    # the time per issue of one VALU kind by a wave at one and at two waves per SIMD
    issue = {f"{k}_ns_{t // 256}w": round(valu_issue(k, t)[0], 4) for k in VALU_KINDS for t in (256, 512)}
    print(json.dumps({"L": a.L, "q": a.q, "flips": a.flips, "reps": a.reps, "max_abs_err_vs_fields": err,
                      "lds_peak_GBps": peak / 1e9, "bytes_per_flip": 40 * a.L, "runs": runs,
                      "valu_issue": issue}))


if __name__ == "__main__":
    main()

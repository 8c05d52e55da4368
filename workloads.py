"""Seeded synthetic workloads shaped like the paper's runs.

This module only generates inputs (temperature ladders, instance shapes,
seeds, arrival times).  It holds none of the method's arithmetic, so both the
GPU path's tests and the CPU oracle can take their inputs from it.

The paper simulates q = 3 rings of L = 512..10240 with 400 uniformly spaced
temperatures (section 5.1 and 5.2); the workloads below keep those shapes
and use geometric ladders, which space the replicas evenly in log T.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 1234


def geometric_ladder(tmin: float, tmax: float, R: int) -> np.ndarray:
    """T_k = tmin (tmax/tmin)^(k/(R-1)), ascending."""
    if R == 1:
        return np.array([tmin], dtype=np.float64)
    k = np.arange(R, dtype=np.float64)
    return tmin * (tmax / tmin) ** (k / (R - 1))


@dataclasses.dataclass
class Instance:
    L: int
    q: int
    sigma: float
    T: np.ndarray
    seed: int
    sweeps: int
    init: int = 0  # 0 uniform random spins, 1 all spins = 1

    @property
    def R(self) -> int:
        return len(self.T)

    @property
    def attempts(self) -> int:
        return self.L * self.R * self.sweeps


def small() -> Instance:
    """L = 64, q = 3, sigma = 0.5, 16 replicas geometric in [0.3, 3], 2000 sweeps."""
    return Instance(64, 3, 0.5, geometric_ladder(0.3, 3.0, 16), SEED, 2000)


def medium() -> Instance:
    """L = 1024, q = 3, sigma = 0.4, 64 replicas geometric in [0.3, 3], 10^4 sweeps."""
    return Instance(1024, 3, 0.4, geometric_ladder(0.3, 3.0, 64), SEED, 10_000)


def large() -> Instance:
    """L = 16384, q = 5, sigma = 0.3, 128 replicas geometric in [0.2, 2.5], ordered start, 2000 sweeps."""
    return Instance(16384, 5, 0.3, geometric_ladder(0.2, 2.5, 128), SEED, 2000, init=1)


def batch_jobs(n_jobs: int = 256, sweeps: int = 1000, R: int = 32, lmin: int = 128, lmax: int = 8192,
               seed: int = SEED) -> list[Instance]:
    """Uneven instances: L log-uniform in [lmin, lmax], q in {2..10}, sigma in [0.1, 1]."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(n_jobs):
        L = int(round(math.exp(rng.uniform(math.log(lmin), math.log(lmax)))))
        q = int(rng.integers(2, 11))
        sigma = float(rng.uniform(0.1, 1.0))
        jobs.append(Instance(L, q, sigma, geometric_ladder(0.2, 3.0, R), seed + j, sweeps))
    return jobs


def serve_stream(rate: float = 50.0, duration: float = 60.0, seed: int = SEED):
    """Poisson arrivals; each job: L log-uniform in [64, 4096], q in {2..8},
    sigma in [0.1, 1], R in {16..64}, sweeps in {500..5000}."""
    rng = np.random.default_rng(seed)
    t, out, j = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        L = int(round(math.exp(rng.uniform(math.log(64), math.log(4096)))))
        q = int(rng.integers(2, 9))
        sigma = float(rng.uniform(0.1, 1.0))
        R = int(rng.integers(16, 65))
        sweeps = int(rng.integers(500, 5001))
        out.append((t, Instance(L, q, sigma, geometric_ladder(0.2, 3.0, R), seed + j, sweeps)))
        j += 1
    return out


def flip_sequence(L: int, q: int, n: int, seed: int = SEED):
    """n single-spin flips with the statistics of accepted ones, from all
    spins in state 0: uniform sites, the old state the site's current one, the
    new state uniform over the other q - 1.  Returns the words
    site | old << 16 | new << 20 (states 0-based) and the final spins."""
    rng = np.random.default_rng(seed)
    s = np.zeros(L, np.int64)
    sites = rng.integers(0, L, n)
    shift = rng.integers(1, q, n) if q > 1 else np.zeros(n, np.int64)
    words = np.empty(n, np.uint32)
    for k in range(n):
        i = sites[k]
        a = s[i]
        b = (a + shift[k]) % q
        words[k] = i | (a << 16) | (b << 20)
        s[i] = b
    return words, s

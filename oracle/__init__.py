"""FP64 CPU oracle for parallel tempering of the 1D long-range q-state Potts ring.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and the
two share no code.  The arithmetic lives in ``orc.c`` (plain C, FP64); this
module builds it with gcc and exposes it through ctypes, plus the exact
enumeration of small rings in :mod:`oracle.enumerate`.

Paper references: section 2 (eqs. 1-7: spins, Hamiltonian, periodic Hurwitz
zeta couplings), section 3 (eqs. 8-9: Metropolis and exchange criteria),
section 4.2 (two-stage even/odd exchange), section 5.1 (eqs. 10-12:
magnetisation and cumulants).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")
_lock = threading.Lock()
_lib = None

BAND = 1e-9  # half-width of the band in which two FP64 evaluations may disagree


def build(force: bool = True) -> str:
    """Compile orc.c into liborc.so with gcc (OpenMP over walkers)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
            _declare(L)
            _lib = L
    return _lib


_d = ctypes.c_double
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def _declare(L):
    L.orc_hurwitz_zeta.restype = _d
    L.orc_hurwitz_zeta.argtypes = [_d, _d]
    L.orc_jstar.restype = ctypes.c_int
    L.orc_jstar.argtypes = [_i32, _d, _p]
    L.orc_philox4x32_10.restype = None
    L.orc_philox4x32_10.argtypes = [_p, _p, _p]
    L.orc_energy.restype = _d
    L.orc_energy.argtypes = [_i32, _p, _p]
    L.orc_energy_ising.restype = _d
    L.orc_energy_ising.argtypes = [_i32, _p, _p]
    L.orc_magnetization.restype = _d
    L.orc_magnetization.argtypes = [_i32, _i32, _p]
    L.orc_pt_create.restype = _p
    L.orc_pt_create.argtypes = [_i32, _i32, _d, _p, _i32, _u64, _i32, _i32]
    L.orc_pt_create_at.restype = _p
    L.orc_pt_create_at.argtypes = [_i32, _i32, _d, _p, _i32, _u64, _i32, _i32, _i32]
    L.orc_pt_free.restype = None
    L.orc_pt_free.argtypes = [_p]
    L.orc_pt_set_threads.argtypes = [_p, _i32]
    L.orc_pt_record_series.argtypes = [_p, _i32]
    L.orc_pt_sweep.argtypes = [_p, _i64]
    L.orc_pt_exchange.argtypes = [_p]
    L.orc_pt_run.argtypes = [_p, _i64, _i32]
    L.orc_pt_set_replay.argtypes = [_p, _i64, _p, _p, _p, _p, _i64, _p, _p, _p, _p]
    L.orc_pt_get_spins.argtypes = [_p, _p]
    L.orc_pt_get_perm.argtypes = [_p, _p]
    L.orc_pt_get_energy.argtypes = [_p, _p]
    L.orc_pt_get_stats.argtypes = [_p, _p, _p, _p, _p, _p, _p]
    L.orc_pt_series_len.restype = _i64
    L.orc_pt_series_len.argtypes = [_p]
    L.orc_pt_get_series.argtypes = [_p, _p, _p]
    L.orc_pt_banded_count.restype = _i64
    L.orc_pt_banded_count.argtypes = [_p]
    L.orc_pt_energy_full.restype = _d
    L.orc_pt_energy_full.argtypes = [_p, _i32]
    L.orc_pt_set_spins.argtypes = [_p, _p]
    L.orc_ising_sweeps.argtypes = [_i32, _p, _p, _d, _u64, _i32, _i64, _i64, _p]


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Couplings (eqs. 4-7), random stream, energies
# --------------------------------------------------------------------------
def hurwitz_zeta(s: float, a: float) -> float:
    """zeta(s, a) = sum_{k>=0} (k + a)^-s (eq. 7)."""
    return lib().orc_hurwitz_zeta(float(s), float(a))


def jstar(L: int, sigma: float) -> np.ndarray:
    """J*(r), r = 0..L-1, from eq. 6 (J*(0) = 0: the self term i = j is excluded)."""
    J = np.zeros(L, dtype=np.float64)
    if lib().orc_jstar(int(L), float(sigma), _ptr(J)) != 0:
        raise ValueError("bad (L, sigma)")
    return J


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return o


def energy(J: np.ndarray, s: np.ndarray) -> float:
    """E = -sum_{i<j} J*(j-i) delta(s_i, s_j) (eq. 2, each pair once), spins 1..q."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    J = np.ascontiguousarray(J, dtype=np.float64)
    return lib().orc_energy(len(s), _ptr(J), _ptr(s))


def energy_ising(J: np.ndarray, sig: np.ndarray) -> float:
    sig = np.ascontiguousarray(sig, dtype=np.int8)
    J = np.ascontiguousarray(J, dtype=np.float64)
    return lib().orc_energy_ising(len(sig), _ptr(J), _ptr(sig))


def magnetization(q: int, s: np.ndarray) -> float:
    """M = (q Nmax / L - 1)/(q - 1) (eq. 10)."""
    s = np.ascontiguousarray(s, dtype=np.uint8)
    return lib().orc_magnetization(len(s), int(q), _ptr(s))


def ising_sweeps(J, sig, beta_ising, seed, walker, sweep0, nsweeps, E):
    """Separately written +-1 spin Metropolis path with the Potts walker's draws."""
    sig = np.ascontiguousarray(sig, dtype=np.int8).copy()
    J = np.ascontiguousarray(J, dtype=np.float64)
    e = ctypes.c_double(E)
    lib().orc_ising_sweeps(len(sig), _ptr(J), _ptr(sig), float(beta_ising), int(seed), int(walker),
                           int(sweep0), int(nsweeps), ctypes.byref(e))
    return sig, e.value


# --------------------------------------------------------------------------
# Parallel tempering
# --------------------------------------------------------------------------
class PT:
    """Oracle parallel-tempering run.  mode 0: direct O(L) dE per attempt;
    mode 1: FP64 field table.  init 0: uniform spins from the walker's
    stream; init 1: all spins 1.  wbase: walker k uses the stream of walker
    wbase + k (to follow selected walkers of a larger run)."""

    def __init__(self, L, q, sigma, T, seed, init=0, mode=0, threads=1, record=False, wbase=0):
        T = np.ascontiguousarray(np.asarray(T, dtype=np.float64))
        self.L, self.q, self.R = int(L), int(q), len(T)
        self.sigma, self.seed = float(sigma), int(seed)
        self.T = T
        self._lib = lib()
        self._h = self._lib.orc_pt_create_at(self.L, self.q, self.sigma, _ptr(T), self.R, self.seed,
                                             int(init), int(mode), int(wbase))
        if not self._h:
            raise ValueError("oracle rejected the arguments")
        self._lib.orc_pt_set_threads(self._h, int(threads))
        self._lib.orc_pt_record_series(self._h, 1 if record else 0)

    def close(self):
        if self._h:
            self._lib.orc_pt_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sweep(self, n=1):
        self._lib.orc_pt_sweep(self._h, int(n))

    def exchange(self):
        self._lib.orc_pt_exchange(self._h)

    def run(self, n, every=1):
        self._lib.orc_pt_run(self._h, int(n), int(every))

    def set_replay(self, met=(), ex=()):
        """met: iterable of (walker, sweep, attempt, decision); ex: (step, stage, slot, decision)."""
        met = np.asarray(list(met), dtype=np.int64).reshape(-1, 4)
        ex = np.asarray(list(ex), dtype=np.int64).reshape(-1, 4)
        cols = [np.ascontiguousarray(met[:, c]) for c in range(3)]
        md = np.ascontiguousarray(met[:, 3].astype(np.int8))
        ecols = [np.ascontiguousarray(ex[:, c]) for c in range(3)]
        ed = np.ascontiguousarray(ex[:, 3].astype(np.int8))
        self._keep = (cols, md, ecols, ed)
        self._lib.orc_pt_set_replay(self._h, len(met), *[_ptr(c) for c in cols], _ptr(md), len(ex),
                                    *[_ptr(c) for c in ecols], _ptr(ed))

    def spins(self) -> np.ndarray:
        out = np.zeros((self.R, self.L), dtype=np.uint8)
        self._lib.orc_pt_get_spins(self._h, _ptr(out))
        return out

    def set_spins(self, s):
        s = np.ascontiguousarray(np.asarray(s, dtype=np.uint8).reshape(self.R, self.L))
        self._lib.orc_pt_set_spins(self._h, _ptr(s))

    def perm(self) -> np.ndarray:
        out = np.zeros(self.R, dtype=np.int32)
        self._lib.orc_pt_get_perm(self._h, _ptr(out))
        return out

    def energies(self) -> np.ndarray:
        out = np.zeros(self.R, dtype=np.float64)
        self._lib.orc_pt_get_energy(self._h, _ptr(out))
        return out

    def energy_full(self, w) -> float:
        return self._lib.orc_pt_energy_full(self._h, int(w))

    def stats(self) -> dict:
        R = self.R
        s6 = np.zeros((6, R)); fa = np.zeros(R, np.int64); fc = np.zeros(R, np.int64)
        xa = np.zeros(max(R - 1, 1), np.int64); xc = np.zeros(max(R - 1, 1), np.int64)
        c3 = np.zeros(3, np.int64)
        self._lib.orc_pt_get_stats(self._h, _ptr(s6), _ptr(fa), _ptr(fc), _ptr(xa), _ptr(xc), _ptr(c3))
        return dict(sumE=s6[0], sumE2=s6[1], sumE4=s6[2], sumM=s6[3], sumM2=s6[4], sumM4=s6[5],
                    flip_att=fa, flip_acc=fc, xchg_att=xa[: R - 1], xchg_acc=xc[: R - 1],
                    samples=int(c3[0]), banded_met=int(c3[1]), banded_ex=int(c3[2]))

    def series(self):
        n = self._lib.orc_pt_series_len(self._h)
        E = np.zeros((n, self.R)); M = np.zeros((n, self.R))
        if n:
            self._lib.orc_pt_get_series(self._h, _ptr(E), _ptr(M))
        return E, M

"""Python binding of libptmi: parallel tempering of the 1D long-range q-state
Potts ring on MI355X (gfx950).

Argument marshalling only: every step of the simulation runs in the HIP
kernels behind the C ABI declared in ``include/ptmi.h``.  PyTorch supplies the
device memory (one workspace tensor per run) and the stream.  There is no CPU
fallback: if the built library is missing this module raises.

Paper: Boer, "GPU-based simulation of the long-range Potts model via parallel
tempering" -- section 2 (eqs. 1-7), section 3 (eqs. 8-9), section 4.2 (two-stage
exchange) and section 5.1 (eqs. 10-12).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libptmi.so")

PT_OK, PT_EINVAL, PT_ENOMEM, PT_EDEVICE, PT_ESTATE = 0, -1, -2, -3, -4
PREC_F64, PREC_F32, PREC_I32 = 0, 1, 2
INIT_RANDOM, INIT_ORDERED = 0, 1
PLACE_AUTO, PLACE_LDS, PLACE_HBM, PLACE_DIRECT = 0, 1, 2, 3
PHASES = ("draw", "chain", "flush", "record", "exchange", "total", "windows", "flushes", "flips", "iters",
          "chain_guess", "chain_correct", "chain_check", "chain_resolve", "chain_redo", "chain_sync")
QMAX = 16
BAND = 1e-9


class PTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"ptmi error {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("init", ctypes.c_int32),
        ("placement", ctypes.c_int32),
        ("threads", ctypes.c_int32),
        ("refresh_every", ctypes.c_int32),
        ("series_capacity", ctypes.c_int32),
        ("event_capacity", ctypes.c_int32),
        ("max_sweeps_per_launch", ctypes.c_int32),
        ("lds_budget", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_size_t),
    ]


class Event(ctypes.Structure):
    _fields_ = [("a", ctypes.c_int64), ("b", ctypes.c_int64), ("c", ctypes.c_int64),
                ("kind", ctypes.c_int32), ("decision", ctypes.c_int32), ("x", ctypes.c_double)]


_P = ctypes.c_void_p


class Obs(ctypes.Structure):
    _fields_ = [
        ("R", ctypes.c_int32), ("q", ctypes.c_int32), ("L", ctypes.c_int32),
        ("sweeps", ctypes.c_int64), ("exchange_steps", ctypes.c_int64), ("samples", ctypes.c_int64),
        ("E", _P), ("M", _P),
        ("sumE", _P), ("sumE2", _P), ("sumE4", _P), ("sumM", _P), ("sumM2", _P), ("sumM4", _P),
        ("flip_att", _P), ("flip_acc", _P), ("xchg_att", _P), ("xchg_acc", _P), ("perm", _P),
        ("n_recheck", ctypes.c_int64), ("n_banded", ctypes.c_int64), ("n_exact_energy", ctypes.c_int64),
        ("n_refresh", ctypes.c_int64), ("n_events_dropped", ctypes.c_int64),
    ]


class JobDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("q", ctypes.c_int32), ("sigma", ctypes.c_double),
                ("T", ctypes.c_void_p), ("R", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("sweeps", ctypes.c_int64), ("exchange_every", ctypes.c_int32), ("init", ctypes.c_int32)]


EXPORTS = [
    "pt_default_options", "pt_workspace_size", "pt_init", "pt_sweep", "pt_exchange", "pt_run",
    "pt_observables", "pt_get_spins", "pt_get_jstar", "pt_get_series", "pt_get_events",
    "pt_get_plan", "pt_get_phase_counters", "pt_reset_stats", "pt_synchronize", "pt_save", "pt_load", "pt_free", "pt_last_error",
    "pt_batch_workspace_size", "pt_batch_create", "pt_batch_run", "pt_batch_observables",
    "pt_batch_get_spins", "pt_batch_shape", "pt_batch_job_stats", "pt_batch_free",
    "pt_server_workspace_size", "pt_server_start", "pt_server_submit", "pt_server_poll", "pt_server_wait", "pt_server_times",
    "pt_server_get_spins", "pt_server_cancel", "pt_server_stop", "pt_run_static",
]
STATIC_SCRATCH_BYTES = 64 << 20

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libptmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with __graft_entry__.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    # PyTorch first: its HIP runtime is then the one the library binds to, so
    # device memory and streams from PyTorch and the library's calls share it
    import torch  # noqa: F401

    L = ctypes.CDLL(path)
    i32, i64, u64, d = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    pp = ctypes.POINTER(ctypes.c_void_p)
    L.pt_default_options.restype = None
    L.pt_default_options.argtypes = [ctypes.POINTER(Options)]
    L.pt_workspace_size.argtypes = [i32, i32, i32, ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
    L.pt_init.argtypes = [pp, i32, i32, d, _P, i32, u64, ctypes.POINTER(Options)]
    L.pt_sweep.argtypes = [_P, i64]
    L.pt_exchange.argtypes = [_P]
    L.pt_run.argtypes = [_P, i64, i32]
    L.pt_observables.argtypes = [_P, ctypes.POINTER(Obs)]
    L.pt_get_spins.argtypes = [_P, _P, _P]
    L.pt_get_jstar.argtypes = [_P, _P]
    L.pt_get_series.argtypes = [_P, _P, _P, i64, ctypes.POINTER(i64)]
    L.pt_get_events.argtypes = [_P, _P, i64, ctypes.POINTER(i64)]
    L.pt_get_phase_counters.argtypes = [_P, _P]
    L.pt_get_plan.argtypes = [_P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.pt_reset_stats.argtypes = [_P]
    L.pt_synchronize.argtypes = [_P]
    L.pt_save.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_size_t)]
    L.pt_load.argtypes = [pp, _P, ctypes.c_size_t, ctypes.POINTER(Options)]
    L.pt_free.argtypes = [_P]
    L.pt_last_error.restype = ctypes.c_char_p
    L.pt_last_error.argtypes = []
    JD, OP, OB = ctypes.POINTER(JobDesc), ctypes.POINTER(Options), ctypes.POINTER(Obs)
    L.pt_batch_workspace_size.argtypes = [JD, i32, OP, ctypes.POINTER(ctypes.c_size_t)]
    L.pt_batch_create.argtypes = [pp, JD, i32, OP]
    L.pt_batch_run.argtypes = [_P]
    L.pt_batch_observables.argtypes = [_P, i32, OB]
    L.pt_batch_get_spins.argtypes = [_P, i32, _P, _P]
    L.pt_batch_shape.argtypes = [_P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.pt_batch_job_stats.argtypes = [_P, i32, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double)]
    L.pt_batch_free.argtypes = [_P]
    L.pt_server_workspace_size.argtypes = [ctypes.c_size_t, i32, ctypes.POINTER(ctypes.c_size_t)]
    L.pt_server_start.argtypes = [pp, ctypes.c_size_t, i32, OP]
    L.pt_server_submit.argtypes = [_P, JD, ctypes.POINTER(i64)]
    L.pt_server_poll.argtypes = [_P, i64, ctypes.POINTER(i32), OB]
    L.pt_server_wait.argtypes = [_P, i64, d, OB]
    L.pt_server_times.argtypes = [_P, i64, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.POINTER(d)]
    L.pt_server_cancel.argtypes = [_P, i64]
    L.pt_server_get_spins.argtypes = [_P, i64, _P, _P]
    L.pt_server_stop.argtypes = [_P]
    L.pt_run_static.argtypes = [i32, i32, d, _P, i32, u64, i64, i32, OP, OB, _P, _P]
    for name in EXPORTS:
        if name != "pt_default_options" and name != "pt_last_error":
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != PT_OK:
        msg = _lib.pt_last_error().decode(errors="replace") if _lib else ""
        raise PTError(status, msg)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _obs_buffers(R):
    arrs = {k: np.zeros(R) for k in ("E", "M", "sumE", "sumE2", "sumE4", "sumM", "sumM2", "sumM4")}
    ints = {k: np.zeros(R, np.int64) for k in ("flip_att", "flip_acc")}
    pairs = {k: np.zeros(max(R - 1, 1), np.int64) for k in ("xchg_att", "xchg_acc")}
    perm = np.zeros(R, np.int32)
    o = Obs()
    for k, v in {**arrs, **ints, **pairs}.items():
        setattr(o, k, _ptr(v))
    o.perm = _ptr(perm)
    return o, arrs, ints, pairs, perm


def _obs_dict(o, arrs, ints, pairs, perm, R):
    out = {**arrs, **ints}
    out.update({k: v[: R - 1] for k, v in pairs.items()})
    out.update(perm=perm, sweeps=o.sweeps, exchange_steps=o.exchange_steps, samples=o.samples,
               n_recheck=o.n_recheck, n_banded=o.n_banded, n_exact_energy=o.n_exact_energy,
               n_refresh=o.n_refresh, n_events_dropped=o.n_events_dropped)
    return out


def _job_desc(job, keep):
    """job: dict or object with L, q, sigma, T, seed, sweeps[, exchange_every, init]."""
    g = (lambda k, d=None: job.get(k, d)) if isinstance(job, dict) else (lambda k, d=None: getattr(job, k, d))
    T = np.ascontiguousarray(np.asarray(g("T"), dtype=np.float64))
    keep.append(T)
    return JobDesc(int(g("L")), int(g("q")), float(g("sigma")), T.ctypes.data, len(T), int(g("seed")),
                   int(g("sweeps")), int(g("exchange_every", 1) or 1), int(g("init", 0) or 0))


def _torch_device_memory(nbytes):
    """Workspace tensor and current stream from PyTorch (device memory and
    stream plumbing only)."""
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to PyTorch; the HIP path has no CPU fallback")
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    return ws, torch.cuda.current_stream().cuda_stream


class Simulation:
    """One parallel-tempering run on the GPU (a pt_ctx).

    L sites, q states, coupling exponent sigma, temperature ladder T (ascending;
    slot k has T[k]), 64-bit seed.  precision PREC_F64 (FP64 field table),
    PREC_F32 (FP32 table + FP64 rechecks) or PREC_I32 (exact int32 table of
    quantised couplings + FP64 rechecks)."""

    def __init__(self, L, q, sigma, T, seed, precision=PREC_F64, init=INIT_RANDOM, threads=0,
                 refresh_every=0, series_capacity=0, event_capacity=0, max_sweeps_per_launch=0,
                 placement=PLACE_AUTO, profile=False, _ctx=None, _ws=None):
        self._lib = load_library()
        self.L, self.q, self.sigma, self.seed = int(L), int(q), float(sigma), int(seed)
        self.T = np.ascontiguousarray(np.asarray(T, dtype=np.float64))
        self.R = len(self.T)
        self.series_capacity = int(series_capacity)
        if _ctx is not None:
            self._ctx, self._ws = _ctx, _ws
            return
        opt = self._options(precision, init, threads, refresh_every, series_capacity, event_capacity,
                            max_sweeps_per_launch, placement)
        opt.profile = 1 if profile else 0
        nbytes = ctypes.c_size_t(0)
        _check(self._lib.pt_workspace_size(self.L, self.q, self.R, ctypes.byref(opt), ctypes.byref(nbytes)))
        self._ws, stream = _torch_device_memory(nbytes.value)
        opt.stream = stream
        opt.workspace = self._ws.data_ptr()
        opt.workspace_bytes = self._ws.numel()
        ctx = ctypes.c_void_p()
        _check(self._lib.pt_init(ctypes.byref(ctx), self.L, self.q, self.sigma, _ptr(self.T), self.R,
                                 self.seed, ctypes.byref(opt)))
        self._ctx = ctx

    def _options(self, precision, init, threads, refresh_every, series_capacity, event_capacity,
                 max_sweeps_per_launch, placement):
        opt = Options()
        self._lib.pt_default_options(ctypes.byref(opt))
        opt.precision, opt.init, opt.threads = int(precision), int(init), int(threads)
        opt.refresh_every, opt.series_capacity = int(refresh_every), int(series_capacity)
        opt.event_capacity, opt.max_sweeps_per_launch = int(event_capacity), int(max_sweeps_per_launch)
        opt.placement = int(placement)
        return opt

    # -- lifecycle ---------------------------------------------------------
    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.pt_free(self._ctx)
            self._ctx = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the hot path --------------------------------------------------------
    def sweep(self, n=1):
        _check(self._lib.pt_sweep(self._ctx, int(n)))

    def exchange(self):
        _check(self._lib.pt_exchange(self._ctx))

    def run(self, n, exchange_every=1):
        _check(self._lib.pt_run(self._ctx, int(n), int(exchange_every)))

    def synchronize(self):
        _check(self._lib.pt_synchronize(self._ctx))

    def reset_stats(self):
        _check(self._lib.pt_reset_stats(self._ctx))

    # -- results -------------------------------------------------------------
    def observables(self) -> dict:
        o, arrs, ints, pairs, perm = _obs_buffers(self.R)
        _check(self._lib.pt_observables(self._ctx, ctypes.byref(o)))
        return _obs_dict(o, arrs, ints, pairs, perm, self.R)

    def plan(self) -> dict:
        """Launch plan chosen at init: placement (PLACE_LDS/HBM/DIRECT), threads, LDS bytes."""
        p, t, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.pt_get_plan(self._ctx, ctypes.byref(p), ctypes.byref(t), ctypes.byref(l)))
        return dict(placement=p.value, threads=t.value, lds_bytes=l.value)

    def phase_counters(self) -> dict:
        """Per-walker phase counters (needs profile=True): cycles per phase and
        counts, each an array [R] by walker, keyed by the names in PHASES."""
        out = np.zeros((self.R, len(PHASES)), np.uint64)
        _check(self._lib.pt_get_phase_counters(self._ctx, _ptr(out)))
        return {name: out[:, k].astype(np.int64) for k, name in enumerate(PHASES)}

    def spins(self):
        """(spins [R][L] by walker, values 1..q; perm [R] slot -> walker)."""
        s = np.zeros((self.R, self.L), np.uint8)
        p = np.zeros(self.R, np.int32)
        _check(self._lib.pt_get_spins(self._ctx, _ptr(s), _ptr(p)))
        return s, p

    def jstar(self) -> np.ndarray:
        out = np.zeros(self.L)
        _check(self._lib.pt_get_jstar(self._ctx, _ptr(out)))
        return out

    def series(self):
        cap = self.series_capacity
        E = np.zeros((max(cap, 1), self.R)); M = np.zeros((max(cap, 1), self.R))
        n = ctypes.c_int64(0)
        _check(self._lib.pt_get_series(self._ctx, _ptr(E), _ptr(M), cap, ctypes.byref(n)))
        return E[: n.value], M[: n.value]

    def events(self, cap=65536):
        buf = (Event * cap)()
        n = ctypes.c_int64(0)
        _check(self._lib.pt_get_events(self._ctx, ctypes.cast(buf, ctypes.c_void_p), cap, ctypes.byref(n)))
        return [(e.kind, e.a, e.b, e.c, e.decision, e.x) for e in buf[: n.value]]

    def save(self) -> bytes:
        n = ctypes.c_size_t(0)
        _check(self._lib.pt_save(self._ctx, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(self._lib.pt_save(self._ctx, ctypes.cast(buf, ctypes.c_void_p), ctypes.byref(n)))
        return buf.raw[: n.value]

    @classmethod
    def load(cls, blob: bytes, **kw):
        lib = load_library()
        import struct

        magic, ver, L, q, R, prec, init, refresh = struct.unpack_from("<IIiiiiii", blob, 0)
        seed, sigma = struct.unpack_from("<Qd", blob, 32)
        T = np.frombuffer(blob, dtype=np.float64, count=R, offset=struct.calcsize("<IIiiiiiiQdqqq"))
        self = cls.__new__(cls)
        opt = Options()
        lib.pt_default_options(ctypes.byref(opt))
        opt.precision, opt.init = prec, init
        opt.series_capacity = int(kw.get("series_capacity", 0))
        opt.refresh_every = int(kw.get("refresh_every", 0))
        nbytes = ctypes.c_size_t(0)
        _check(lib.pt_workspace_size(L, q, R, ctypes.byref(opt), ctypes.byref(nbytes)))
        ws, stream = _torch_device_memory(nbytes.value)
        opt.stream, opt.workspace, opt.workspace_bytes = stream, ws.data_ptr(), ws.numel()
        ctx = ctypes.c_void_p()
        raw = ctypes.create_string_buffer(blob, len(blob))
        _check(lib.pt_load(ctypes.byref(ctx), ctypes.cast(raw, ctypes.c_void_p), len(blob), ctypes.byref(opt)))
        Simulation.__init__(self, L, q, sigma, T, seed, _ctx=ctx, _ws=ws,
                            series_capacity=opt.series_capacity)
        return self


def run_static(L, q, sigma, T, seed, sweeps, exchange_every=1, precision=PREC_F64, init=INIT_RANDOM,
               threads=0, placement=PLACE_AUTO, max_sweeps_per_launch=0, event_capacity=0):
    """pt_run_static: pt_init + pt_run + pt_observables + pt_get_spins in one
    call that allocates no device memory (the state lives in the library's
    static device buffer).  Runs on PyTorch's current stream.  Returns
    (observables dict, spins [R][L] by walker with values 1..q, perm)."""
    import torch

    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible to PyTorch; the HIP path has no CPU fallback")
    T = np.ascontiguousarray(np.asarray(T, dtype=np.float64))
    R = len(T)
    opt = Options()
    lib.pt_default_options(ctypes.byref(opt))
    opt.precision, opt.init, opt.threads, opt.placement = int(precision), int(init), int(threads), int(placement)
    opt.max_sweeps_per_launch, opt.event_capacity = int(max_sweeps_per_launch), int(event_capacity)
    opt.stream = torch.cuda.current_stream().cuda_stream
    o, arrs, ints, pairs, perm = _obs_buffers(R)
    spins = np.zeros((R, int(L)), np.uint8)
    perm2 = np.zeros(R, np.int32)
    _check(lib.pt_run_static(int(L), int(q), float(sigma), _ptr(T), R, int(seed), int(sweeps), int(exchange_every),
                             ctypes.byref(opt), ctypes.byref(o), _ptr(spins), _ptr(perm2)))
    return _obs_dict(o, arrs, ints, pairs, perm, R), spins, perm2


class Batch:
    """Many independent runs of uneven size in one persistent launch (pt_batch).

    jobs: list of dicts/objects with L, q, sigma, T, seed, sweeps, and optional
    exchange_every (default 1) and init.  threads / lds_budget set the walker
    workgroup shape (0 = library default)."""

    def __init__(self, jobs, precision=PREC_F64, threads=0, lds_budget=0):
        self._lib = load_library()
        keep = []
        self.jobs = list(jobs)
        arr = (JobDesc * len(self.jobs))(*[_job_desc(j, keep) for j in self.jobs])
        opt = Options()
        self._lib.pt_default_options(ctypes.byref(opt))
        opt.precision, opt.threads, opt.lds_budget = int(precision), int(threads), int(lds_budget)
        nbytes = ctypes.c_size_t(0)
        _check(self._lib.pt_batch_workspace_size(arr, len(self.jobs), ctypes.byref(opt), ctypes.byref(nbytes)))
        self._ws, stream = _torch_device_memory(nbytes.value)
        opt.stream, opt.workspace, opt.workspace_bytes = stream, self._ws.data_ptr(), self._ws.numel()
        h = ctypes.c_void_p()
        _check(self._lib.pt_batch_create(ctypes.byref(h), arr, len(self.jobs), ctypes.byref(opt)))
        self._h = h
        self.R = [len(np.asarray(k["T"] if isinstance(k, dict) else k.T)) for k in self.jobs]

    def run(self):
        _check(self._lib.pt_batch_run(self._h))

    def shape(self):
        w, t, l = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(self._lib.pt_batch_shape(self._h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(l)))
        return dict(workgroups=w.value, threads=t.value, lds_bytes=l.value)

    def job_stats(self, j) -> dict:
        """Placement of job j's table (PLACE_*) and, after run(), the device
        wall clock (s) when its set-up began and when its last walker ended."""
        p, t0, t1 = ctypes.c_int32(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.pt_batch_job_stats(self._h, int(j), ctypes.byref(p), ctypes.byref(t0), ctypes.byref(t1)))
        return dict(placement=p.value, start=t0.value, end=t1.value)

    def observables(self, j) -> dict:
        R = self.R[j]
        o, arrs, ints, pairs, perm = _obs_buffers(R)
        _check(self._lib.pt_batch_observables(self._h, int(j), ctypes.byref(o)))
        return _obs_dict(o, arrs, ints, pairs, perm, R)

    def spins(self, j):
        R = self.R[j]
        L = int(self.jobs[j]["L"] if isinstance(self.jobs[j], dict) else self.jobs[j].L)
        s = np.zeros((R, L), np.uint8)
        p = np.zeros(R, np.int32)
        _check(self._lib.pt_batch_get_spins(self._h, int(j), _ptr(s), _ptr(p)))
        return s, p

    def close(self):
        if getattr(self, "_h", None):
            self._lib.pt_batch_free(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous batching: a persistent launch that takes jobs while it runs
    (pt_server).  Jobs wait until their state fits in the device arena.  The
    launch stays resident until stop(): do not call torch.cuda.synchronize()
    (a device-wide wait) while a server runs."""

    def __init__(self, arena_bytes=1 << 30, max_jobs=8192, precision=PREC_F64, threads=0, lds_budget=0):
        self._lib = load_library()
        opt = Options()
        self._lib.pt_default_options(ctypes.byref(opt))
        opt.precision, opt.threads, opt.lds_budget = int(precision), int(threads), int(lds_budget)
        # the device arena and control words come from PyTorch
        nbytes = ctypes.c_size_t(0)
        _check(self._lib.pt_server_workspace_size(int(arena_bytes), int(max_jobs), ctypes.byref(nbytes)))
        self._ws, _ = _torch_device_memory(nbytes.value)
        opt.workspace, opt.workspace_bytes = self._ws.data_ptr(), self._ws.numel()
        h = ctypes.c_void_p()
        _check(self._lib.pt_server_start(ctypes.byref(h), int(arena_bytes), int(max_jobs), ctypes.byref(opt)))
        self._h = h
        self._R, self._L = {}, {}

    def submit(self, job) -> int:
        keep = []
        d = _job_desc(job, keep)
        jid = ctypes.c_int64()
        _check(self._lib.pt_server_submit(self._h, ctypes.byref(d), ctypes.byref(jid)))
        self._R[jid.value], self._L[jid.value] = d.R, d.L
        return jid.value

    def poll(self, jid):
        R = self._R[jid]
        o, arrs, ints, pairs, perm = _obs_buffers(R)
        done = ctypes.c_int32()
        _check(self._lib.pt_server_poll(self._h, int(jid), ctypes.byref(done), ctypes.byref(o)))
        return _obs_dict(o, arrs, ints, pairs, perm, R) if done.value else None

    def wait(self, jid, timeout=600.0) -> dict:
        R = self._R[jid]
        o, arrs, ints, pairs, perm = _obs_buffers(R)
        _check(self._lib.pt_server_wait(self._h, int(jid), float(timeout), ctypes.byref(o)))
        return _obs_dict(o, arrs, ints, pairs, perm, R)

    def cancel(self, jid) -> bool:
        """Drop a job still waiting in the host queue: True; False if it was
        already admitted (it then runs to its end)."""
        st = self._lib.pt_server_cancel(self._h, int(jid))
        if st == PT_ESTATE:
            return False
        _check(st)
        return True

    def times(self, jid):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(self._lib.pt_server_times(self._h, int(jid), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def spins(self, jid):
        s = np.zeros((self._R[jid], self._L[jid]), np.uint8)
        p = np.zeros(self._R[jid], np.int32)
        _check(self._lib.pt_server_get_spins(self._h, int(jid), _ptr(s), _ptr(p)))
        return s, p

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(self._lib.pt_server_stop(h))
            self._ws = None  # the launch has ended: the arena goes back to PyTorch

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass

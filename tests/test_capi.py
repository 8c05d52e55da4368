"""Host-side checks of the C ABI: the built library loads and exports every
entry point declared in include/ptmi.h (no compute calls: no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    text = open(os.path.join(ROOT, "include", "ptmi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pt_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for required in ["pt_init", "pt_sweep", "pt_exchange", "pt_observables", "pt_run", "pt_get_spins",
                     "pt_save", "pt_load", "pt_free", "pt_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1308_5426_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(pkg.EXPORTS) == declared_entry_points()


def test_host_only_calls():
    """Calls that touch no device: defaults, workspace sizing, argument errors."""
    import paper_1308_5426_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = pkg.load_library()
    opt = pkg.Options()
    lib.pt_default_options(ctypes.byref(opt))
    assert opt.precision == pkg.PREC_F64 and opt.init == pkg.INIT_RANDOM
    n = ctypes.c_size_t(0)
    assert lib.pt_workspace_size(1024, 3, 64, ctypes.byref(opt), ctypes.byref(n)) == 0
    assert n.value > 1024 * 2 * 64 * 8  # rows 0 and 1 of q = 3 (the last row is implicit)
    opt.precision = pkg.PREC_F32
    n32 = ctypes.c_size_t(0)
    assert lib.pt_workspace_size(1024, 3, 64, ctypes.byref(opt), ctypes.byref(n32)) == 0
    assert n32.value < n.value
    opt.precision = pkg.PREC_I32
    ni = ctypes.c_size_t(0)
    assert lib.pt_workspace_size(1024, 3, 64, ctypes.byref(opt), ctypes.byref(ni)) == 0
    assert ni.value == n32.value  # 4-byte table entries either way
    opt.placement = pkg.PLACE_DIRECT  # direct sums keep no table: no int32 form
    ctx = ctypes.c_void_p()
    Tl = (ctypes.c_double * 2)(1.0, 2.0)
    assert lib.pt_init(ctypes.byref(ctx), 10, 3, 0.5, ctypes.cast(Tl, ctypes.c_void_p), 2, 1,
                       ctypes.byref(opt)) == pkg.PT_EINVAL
    opt.placement = pkg.PLACE_AUTO
    opt.precision = 3
    assert lib.pt_init(ctypes.byref(ctx), 10, 3, 0.5, ctypes.cast(Tl, ctypes.c_void_p), 2, 1,
                       ctypes.byref(opt)) == pkg.PT_EINVAL
    opt.precision = pkg.PREC_F32
    assert lib.pt_workspace_size(1, 3, 64, ctypes.byref(opt), ctypes.byref(n)) == pkg.PT_EINVAL
    assert lib.pt_workspace_size(10, 17, 64, ctypes.byref(opt), ctypes.byref(n)) == pkg.PT_EINVAL
    assert b"bad sizes" in lib.pt_last_error()
    ctx = ctypes.c_void_p()
    T = (ctypes.c_double * 2)(2.0, 1.0)
    assert lib.pt_init(ctypes.byref(ctx), 10, 3, 0.5, ctypes.cast(T, ctypes.c_void_p), 2, 1, None) == pkg.PT_EINVAL
    assert b"ascending" in lib.pt_last_error()
    assert lib.pt_sweep(None, 1) == pkg.PT_EINVAL
    assert lib.pt_server_cancel(None, 0) == pkg.PT_EINVAL
    assert lib.pt_batch_job_stats(None, 0, None, None, None) == pkg.PT_EINVAL


def test_probe_library_exports():
    import paper_1308_5426_amd as pkg

    path = os.path.join(os.path.dirname(pkg.LIB_PATH), "libptmi_probe.so")
    if not os.path.exists(path):
        pytest.skip("probe library not built")
    lib = ctypes.CDLL(path)
    text = open(os.path.join(ROOT, "include", "ptmi_probe.h")).read()
    for name in re.findall(r"\b(ptmi_[a-z_]+)\s*\(", text):
        assert hasattr(lib, name)


def _checkpoint(L, q, R, spins, perm, prec=0, init=0, T=None, sigma=0.5):
    """A checkpoint buffer in the library's layout: header, T, spins (0-based),
    perm, six moment sums and four counter arrays per slot."""
    import struct

    import numpy as np

    hdr = struct.pack("<IIiiiiiiQdqqq", 0x50544D49, 1, L, q, R, prec, init, 0, 1234, sigma, 0, 0, 0)
    T = (np.linspace(1.0, 2.0, R) if T is None else np.asarray(T, float)).astype("<f8").tobytes()
    body = (np.asarray(spins, np.uint8).tobytes() + np.asarray(perm, "<i4").tobytes()
            + np.zeros(6 * R, "<f8").tobytes() + np.zeros(4 * R, "<i8").tobytes())
    return hdr + T + body


@pytest.mark.parametrize("case", ["valid", "spin_equal_q", "spin_255", "perm_duplicate", "perm_range",
                                  "bad_sizes", "short"])
def test_load_rejects_corrupt_checkpoint(case):
    """pt_load checks the buffer on the host before any device call: a spin
    outside 0..q-1 or a perm that is not a permutation is PT_EINVAL."""
    import numpy as np

    import paper_1308_5426_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = pkg.load_library()
    L, q, R = 16, 3, 4
    spins = np.zeros((R, L), np.uint8)
    perm = np.arange(R)
    if case == "spin_equal_q":
        spins[2, 7] = q
    elif case == "spin_255":
        spins[0, 0] = 255
    elif case == "perm_duplicate":
        perm = np.array([0, 1, 1, 3])
    elif case == "perm_range":
        perm = np.array([0, 1, 2, 4])
    blob = _checkpoint(L, q, R, spins, perm)
    if case == "bad_sizes":
        blob = _checkpoint(L, 99, R, spins, perm)
    if case == "short":
        blob = blob[:-8]
    raw = ctypes.create_string_buffer(blob, len(blob))
    ctx = ctypes.c_void_p()
    st = lib.pt_load(ctypes.byref(ctx), ctypes.cast(raw, ctypes.c_void_p), len(blob), None)
    if case == "valid":  # passes the host checks: loads on a GPU, fails at the device without one
        assert st in (pkg.PT_OK, pkg.PT_EDEVICE), lib.pt_last_error()
        if st == pkg.PT_OK:
            assert lib.pt_free(ctx) == pkg.PT_OK
        return
    assert st == pkg.PT_EINVAL, lib.pt_last_error()
    assert not ctx.value


@pytest.mark.parametrize("bad", ["T_nan", "T_inf", "T_zero", "sigma_nan", "sigma_inf"])
def test_non_finite_inputs_are_refused_on_the_host(bad):
    """NaN or infinite temperatures or sigma, given directly or inside a
    checkpoint, are refused with PT_EINVAL before any device call."""
    import numpy as np

    import paper_1308_5426_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = pkg.load_library()
    L, q, R = 16, 3, 4
    T = np.linspace(1.0, 2.0, R)
    sigma = 0.5
    if bad == "T_nan":
        T[2] = np.nan
    elif bad == "T_inf":
        T[3] = np.inf
    elif bad == "T_zero":
        T[0] = 0.0
    elif bad == "sigma_nan":
        sigma = float("nan")
    else:
        sigma = float("inf")
    ctx = ctypes.c_void_p()
    Tc = np.ascontiguousarray(T)
    st = lib.pt_init(ctypes.byref(ctx), L, q, ctypes.c_double(sigma), Tc.ctypes.data_as(ctypes.c_void_p), R, 1, None)
    assert st == pkg.PT_EINVAL and not ctx.value, lib.pt_last_error()
    blob = _checkpoint(L, q, R, np.zeros((R, L), np.uint8), np.arange(R), T=T, sigma=sigma)
    raw = ctypes.create_string_buffer(blob, len(blob))
    st = lib.pt_load(ctypes.byref(ctx), ctypes.cast(raw, ctypes.c_void_p), len(blob), None)
    assert st == pkg.PT_EINVAL and not ctx.value, lib.pt_last_error()


def test_run_static_rejects_on_the_host():
    """pt_run_static refuses bad arguments, a caller workspace and a state beyond
    its static buffer before any device call (no GPU needed)."""
    import numpy as np

    import paper_1308_5426_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = pkg.load_library()
    T = np.linspace(0.5, 2.0, 128)
    Tp = T.ctypes.data_as(ctypes.c_void_p)
    assert lib.pt_run_static(1, 3, 0.5, Tp, 4, 1, 1, 1, None, None, None, None) == pkg.PT_EINVAL
    assert lib.pt_run_static(64, 3, 0.5, Tp, 4, 1, -1, 1, None, None, None, None) == pkg.PT_EINVAL
    opt = pkg.Options()
    lib.pt_default_options(ctypes.byref(opt))
    opt.workspace, opt.workspace_bytes = 4096, 1 << 20
    assert lib.pt_run_static(64, 3, 0.5, Tp, 4, 1, 1, 1, ctypes.byref(opt), None, None, None) == pkg.PT_EINVAL
    assert b"no workspace" in lib.pt_last_error()
    # FP64 table state of 128 walkers x 65535 sites x 16 states: far beyond 64 MiB
    assert lib.pt_run_static(65535, 16, 0.5, Tp, 128, 1, 1, 1, None, None, None, None) == pkg.PT_EINVAL
    assert b"static buffer" in lib.pt_last_error()
    assert pkg.STATIC_SCRATCH_BYTES == 64 << 20

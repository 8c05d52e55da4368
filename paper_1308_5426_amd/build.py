"""Build the gfx950 HIP library libptmi.so in-tree with hipcc.

The library is compiled from several sources in parallel (the host runtime and
C ABI in csrc/ptmi.hip, the kernel variants of each field-table precision in
csrc/kernels_<prec>.hip) and linked into one shared object; the LDS bandwidth
probe is a library of its own."""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["ptmi.hip", "kernels_f64.hip", "kernels_f32.hip", "kernels_i32.hip"]
LIB = os.path.join(HERE, "libptmi.so")
PROBE_SRC = os.path.join(CSRC, "lds_probe.hip")
PROBE_LIB = os.path.join(HERE, "libptmi_probe.so")
OBJ_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("PTMI_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]
INCLUDES = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)


def _object(src, verbose):
    obj = os.path.join(OBJ_DIR, os.path.splitext(src)[0] + ".o")
    _run([hipcc(), *FLAGS, *INCLUDES, "-c", os.path.join(CSRC, src), "-o", obj], verbose)
    return obj


def _link(objs, lib, verbose):
    tmp = lib + ".tmp%d" % os.getpid()
    _run([hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp], verbose)
    os.replace(tmp, lib)


def _probe(verbose):
    tmp = PROBE_LIB + ".tmp%d" % os.getpid()
    _run([hipcc(), *FLAGS, "-shared", *INCLUDES, PROBE_SRC, "-o", tmp], verbose)
    os.replace(tmp, PROBE_LIB)


def build(verbose: bool = False) -> str:
    """Compile csrc/ptmi.hip and csrc/kernels_*.hip (with the headers they
    include) into libptmi.so, and the LDS bandwidth probe into libptmi_probe.so."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES) + 1) as ex:
        probe = ex.submit(_probe, verbose)
        objs = [f.result() for f in [ex.submit(_object, s, verbose) for s in SOURCES]]
        _link(objs, LIB, verbose)
        probe.result()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

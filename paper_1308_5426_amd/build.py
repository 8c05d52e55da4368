"""Build the gfx950 HIP library libptmi.so in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "ptmi.hip")
LIB = os.path.join(HERE, "libptmi.so")
PROBE_SRC = os.path.join(HERE, "csrc", "lds_probe.hip")
PROBE_LIB = os.path.join(HERE, "libptmi_probe.so")
ARCH = os.environ.get("PTMI_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found")
    return exe


def _compile(src, lib, verbose):
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"), src, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    """Compile csrc/ptmi.hip (and the headers it includes) into libptmi.so, and
    the LDS bandwidth probe into libptmi_probe.so."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(2) as ex:
        for f in [ex.submit(_compile, SRC, LIB, verbose), ex.submit(_compile, PROBE_SRC, PROBE_LIB, verbose)]:
            f.result()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

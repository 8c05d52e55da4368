"""The host runtime under AddressSanitizer and UndefinedBehaviorSanitizer:
csrc/ptmi.hip is compiled with both on its host code only (the GPU code is
built as usual), linked with the library's kernel objects and a C++ driver
that makes every host-side call of the C ABI (defaults, sizing, argument
refusals, corrupt checkpoints), and run without a GPU; the build aborts on the
first report.  CPU only; needs the kernel objects of a prior build."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
PKG = os.path.join(ROOT, "paper_1308_5426_amd")


def test_host_runtime_is_clean_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    kobj = [os.path.join(PKG, "_build", f"kernels_{p}.o") for p in ("f64", "f32", "i32")]
    if not all(os.path.exists(o) for o in kobj):
        pytest.skip("kernel objects not built")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", *san, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc")]
    rt = str(tmp_path / "ptmi.o")
    drv = str(tmp_path / "driver.o")
    exe = str(tmp_path / "capi_sanitize")
    for src, obj in ((os.path.join(PKG, "csrc", "ptmi.hip"), rt), (os.path.join(HERE, "capi_sanitize_driver.cpp"), drv)):
        subprocess.run([hipcc, *flags, "-c", src, "-o", obj], check=True, capture_output=True, timeout=300)
    subprocess.run([hipcc, *flags, drv, rt, *kobj, "-o", exe], check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")

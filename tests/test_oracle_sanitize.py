"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: a C
driver calls every entry point of oracle/orc.c on small and edge cases (L = 2
and 3, q up to 16, one replica, several threads, replayed decisions, spins
set from outside) in a build that aborts on the first report.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "orc_sanitize")
    cmd = [gcc, "-O1", "-g", "-std=c11", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "oracle"),
           os.path.join(HERE, "orc_sanitize_driver.c"), os.path.join(ROOT, "oracle", "orc.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=240)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="3")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip().endswith("ok")

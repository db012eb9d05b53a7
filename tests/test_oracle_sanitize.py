"""The CPU oracle's C under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/sanitize_oracle.c drives every entry point on small and degenerate
grids (down to 1x1x1, whose links all wrap onto the site itself), with two
OpenMP threads; any report aborts the run.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_is_clean_under_sanitizers(tmp_path):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no gcc")
    exe = tmp_path / "sanitize_oracle"
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", str(exe),
           os.path.join(HERE, "sanitize_oracle.c"),
           os.path.join(ROOT, "oracle", "lbm81_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in r.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", \
        (r.returncode, r.stdout[-500:], r.stderr[-3000:])

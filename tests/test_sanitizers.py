"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host only): a driver
builds plain and bisulfite indexes, seeds random reads with N bases by both oracle methods (with
re-seeding and the k-mer shortcut) and runs the rescue prefilter; any sanitizer report fails."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        subprocess.check_call(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                               "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "sanitize_driver.c"),
                               os.path.join(ROOT, "oracle", "oracle.c"), "-lm"])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
                   OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "seeds" in r.stdout and "rescue" in r.stdout

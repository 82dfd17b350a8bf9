"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/oracle_sanitize_driver.c calls it on random small scenes with random
parameters; any out-of-bounds access, overflow or other undefined behaviour
aborts the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_sanitizers():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "drv")
        subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "oracle"),
                        os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
                        os.path.join(ROOT, "oracle", "sil_ref.c"), "-o", exe], check=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.startswith("ok"), r.stdout

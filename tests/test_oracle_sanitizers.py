"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer.

oracle.c is compiled with gcc together with tests/oracle_sanitize_main.c,
which calls every entry point on small grids (both lattices, periodic and
zero-gradient axes, both anomaly differences, a general caloric law,
degenerate one-node axes).  Any out-of-bounds access, use after free, leak or
undefined arithmetic ends the run with a non-zero status.  CPU only.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitized")
        cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), "-o", exe,
               os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
               "-lm"]
        subprocess.check_call(cmd)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "runtime error" not in r.stderr, r.stderr
        assert "all checks passed" in r.stdout

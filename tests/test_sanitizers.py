"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

gcc builds ``tests/sanitize_driver.c`` (which includes ``oracle/wo_oracle.c``)
with ``-fsanitize=address,undefined`` and runs it: every route and batching
rule on small seeded instances, threaded against single-plan evaluation, and
the route functions on edge inputs.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    subprocess.check_call(["gcc", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-O1", "-g",
                           "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined",
                           os.path.join(HERE, "sanitize_driver.c"), "-o", exe, "-lpthread"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]

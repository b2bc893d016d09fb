"""The CPU oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer.

gcc builds ``tests/sanitize_driver.c`` (which includes ``oracle/wo_oracle.c``)
with ``-fsanitize=address,undefined`` and runs it: every route and batching
rule on small seeded instances, threaded against single-plan evaluation, and
the route functions on edge inputs.  hipcc builds the library with the
sanitizers on its host code only, and the C-ABI tests that need no GPU run
against it.  Any sanitizer report fails the test."""
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


def _clang_asan_runtime():
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.mark.skipif(_clang_asan_runtime() is None, reason="needs the clang AddressSanitizer runtime")
def test_host_library_under_sanitizers(tmp_path):
    # the library's host code (argument checks, descriptor validation and
    # packing, checkpoint headers, the no-allocation scratch checks) built
    # with AddressSanitizer and UndefinedBehaviorSanitizer, driven by the
    # C-ABI tests that need no GPU; any report fails the test
    import sys
    root = os.path.dirname(HERE)
    sys.path.insert(0, root)
    from paper_2110_13693_amd import build
    so = build.build(out=str(tmp_path / "libwo_san.so"), sanitize=True)
    logs = tmp_path / "san"
    env = dict(os.environ, WO_LIBRARY=so, LD_PRELOAD=_clang_asan_runtime(),
               ASAN_OPTIONS="detect_leaks=0:detect_odr_violation=0:log_path=%s" % logs,
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:log_path=%s" % logs)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(HERE, "test_abi_cpu.py")], capture_output=True, text=True, env=env,
                       cwd=root, timeout=600)
    reports = [open(p).read() for p in map(str, tmp_path.iterdir()) if os.path.basename(p).startswith("san")]
    assert not reports, reports[0][:4000]
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]

"""Build ``libwo.so`` (the C-ABI library with the gfx950 kernels) in-tree.

Every source is compiled by hipcc for gfx950 only; packed FP32 instructions
are disabled (``-packed-fp32-ops``).  ``build()`` always recompiles.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libwo.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["wo_api.cpp", "eval.hip", "surrogate.hip", "surrogate_api.cpp", "search.hip", "search_api.cpp",
           "firstfit.hip", "kmeans.hip", "peaks.hip", "aisle.hip", "svm.hip"]
ARCH = "gfx950"
NO_CONTRACT = {"svm.hip", "aisle.hip"}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-command-line-argument", "-I" + CSRC]


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (the
# device code is built as usual); the program that loads such a library must
# have the sanitizer runtime preloaded
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]


def build(verbose: bool = False, out: str = OUT, sanitize: bool = False) -> str:
    """Compile every source and link ``out``; ``sanitize`` adds the host
    sanitizers (into a separate build folder)."""
    build_dir = BUILD_DIR + ("_san" if sanitize else "")
    os.makedirs(build_dir, exist_ok=True)
    cc = hipcc()
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        # IEEE double one operation at a time where the results must equal
        # the oracle's bit for bit
        extra = ["-ffp-contract=off"] if src in NO_CONTRACT else []
        cmd = [cc] + COMMON + extra + (SANITIZE_HOST if sanitize else []) + \
            ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        log, _ = p.communicate()
        text = log.decode(errors="replace")
        # the host pass does not know the packed-fp32 feature: harmless, filter it
        text = "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(text + "\n")
        elif verbose and text.strip():
            print(text)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call([cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] +
                          (SANITIZE_HOST if sanitize else []) + objs)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

"""Host-side sanitizer check (CPU only): builds the oracle with gcc and the
library's host code with hipcc, both with AddressSanitizer and
UndefinedBehaviorSanitizer (the device code is built as usual: sanitizers
apply to the host pass only), then runs the oracle's pin tests and the C ABI's
host tests against those builds, each sanitizer runtime preloaded into its own
pytest process.  Any sanitizer report fails the run.

    python -m paper_2002_12921_amd.sanitize
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

from . import build as libbuild

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
OUT = os.path.join(HERE, "_build", "san")
SAN = ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=undefined"]


def build_oracle() -> str:
    path = os.path.join(OUT, "libvegas_oracle_san.so")
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", *SAN, "-ffp-contract=off",
                           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-o", path,
                           os.path.join(ROOT, "oracle", "vegas_oracle.c"), "-lm"])
    return path


def build_library(jobs: int = 8) -> str:
    """libvegas with the host pass instrumented (each -fsanitize= after
    -Xarch_host, so the device code is untouched)."""
    host = []
    for f in SAN + ["-fno-omit-frame-pointer"]:
        host += ["-Xarch_host", f]
    return libbuild.build(out=os.path.join(OUT, "libvegas_gfx950_san.so"), objdir=os.path.join(OUT, "obj"),
                          extra=host, link_extra=host, jobs=jobs)


def _clang_asan_runtime() -> str:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("clang's AddressSanitizer runtime not found under /opt/rocm/llvm")
    return hits[-1]


def _gcc_asan_runtime() -> str:
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


def run() -> int:
    os.makedirs(OUT, exist_ok=True)
    oracle_so = build_oracle()
    lib_so = build_library()
    base = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    oracle_tests = sorted(glob.glob(os.path.join(ROOT, "tests", "test_oracle_*.py")))
    runs = [
        ("oracle pins (gcc ASan+UBSan)", dict(base, LD_PRELOAD=_gcc_asan_runtime(), VEGAS_ORACLE_LIB=oracle_so),
         oracle_tests),
        ("C ABI host tests (clang ASan+UBSan, host pass)", dict(base, LD_PRELOAD=_clang_asan_runtime(), VEGAS_LIB=lib_so),
         [os.path.join(ROOT, "tests", "test_capi_host.py")]),
    ]
    rc = 0
    for name, env, tests in runs:
        print(f"== {name}", flush=True)
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-m", "not gpu", "-p", "no:cacheprovider", *tests],
                           env=env, cwd=ROOT)
        rc = rc or r.returncode
    return rc


if __name__ == "__main__":
    sys.exit(run())

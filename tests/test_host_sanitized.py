"""The host-side tests again, against libcfc_san.so: the library's host C++
(graph canonicalisation, hierarchy setup, elimination, the counter-based
draws, the C ABI's argument checks) built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only) and run in a child interpreter
with the ASan runtime preloaded.  Any sanitizer report fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_LIB = os.path.join(ROOT, "paper_1607_02955_amd", "libcfc_san.so")


def asan_runtime():
    r = subprocess.run([os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"),
                        "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isfile(path) else None


def stale():
    """The sanitized build is missing or older than a source or header."""
    if not os.path.exists(SAN_LIB):
        return True
    t = os.path.getmtime(SAN_LIB)
    srcs = [os.path.join(d, f) for d in (os.path.join(ROOT, "paper_1607_02955_amd", "csrc"),
                                          os.path.join(ROOT, "include")) for f in os.listdir(d)]
    return any(os.path.getmtime(f) > t for f in srcs)


def test_host_suite_under_asan_and_ubsan():
    if stale():
        sys.path.insert(0, ROOT)
        from paper_1607_02955_amd import build as B
        B.build(verbose=False, sanitize=True)
    rt = asan_runtime()
    if rt is None:
        pytest.skip("the ASan runtime of hipcc's clang is not installed")
    env = dict(os.environ, CFC_LIB_PATH=SAN_LIB, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_host.py"),
                        "-q", "-m", "not gpu", "-p", "no:cacheprovider", "-x"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    print(tail)
    assert "AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert r.returncode == 0, tail
    assert " passed" in r.stdout

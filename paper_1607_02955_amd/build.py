"""Build libcfc.so in-tree with hipcc for gfx950.

Every source under csrc/ is compiled as HIP (hipcc -x hip) with packed-FP32
instructions disabled, then linked into paper_1607_02955_amd/libcfc.so.
Run as ``python -m paper_1607_02955_amd.build`` or through
``__graft_entry__.build()``.

``build(sanitize=True)`` (``python -m paper_1607_02955_amd.build --sanitize``)
builds libcfc_san.so instead: the same sources with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code only (each -fsanitize flag
behind -Xarch_host; the device code is not instrumented), for running the
host-side tests under the sanitizers (tests/test_host_sanitized.py).
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libcfc.so")
OUT_SAN = os.path.join(HERE, "libcfc_san.so")
BUILD = os.path.join(os.path.dirname(HERE), "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("CFC_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-command-line-argument"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.cpp")) + glob.glob(os.path.join(CSRC, "*.hip")))


SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _flags(sanitize):
    return [f for f in FLAGS if f != "-O3"] + SAN_FLAGS if sanitize else FLAGS


def _compile(src, sanitize=False):
    obj = os.path.join(BUILD, os.path.basename(src) + (".san.o" if sanitize else ".o"))
    cmd = [HIPCC, "-x", "hip", *_flags(sanitize), "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
    return obj, msg


def build(verbose=True, jobs=None, sanitize=False):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 4)))
    objs = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, msg in ex.map(lambda f: _compile(f, sanitize), srcs):
            objs.append(obj)
            if msg and verbose:
                print(msg, file=sys.stderr)
    out = OUT_SAN if sanitize else OUT
    tmp = out + ".tmp"
    cmd = [HIPCC, *_flags(sanitize), "-shared", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}", file=sys.stderr)
    return out


if __name__ == "__main__":
    build(sanitize="--sanitize" in sys.argv[1:])

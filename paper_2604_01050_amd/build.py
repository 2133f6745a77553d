"""Build libsbqa.so (HIP kernels + C ABI runtime) for gfx950 with hipcc.

Usage: python -m paper_2604_01050_amd.build   (or build.build()).
Objects go to <repo>/_build/, the library to paper_2604_01050_amd/libsbqa.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(PKG, "libsbqa.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed fp32 instructions are disabled on purpose: hand-written or generated
# v_pk_{add,mul,fma}_f32 are avoided on this target. MFMA accumulators and
# results are allocated in ordinary VGPRs (gfx950 reads and writes both
# register halves): with accumulation registers the allocator rotated the
# dense step's accumulators through copies every loop iteration, each copy
# waiting on an MFMA.
COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH, "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
          "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, *COMMON, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every source under csrc/ and link libsbqa.so. Always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    jobs = jobs or min(8, len(srcs))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, OUT)
    if verbose:
        print("built", OUT)
    return OUT


# Host sanitizers for the test driver tests/sanitize/host_checks.cpp: only
# the host part of each source is instrumented (each -fsanitize= behind
# -Xarch_host); device code is built as above.
SANITIZERS = {
    "asan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"],
    "tsan": ["-Xarch_host", "-fsanitize=thread"],
}


def build_sanitized(kind: str, verbose: bool = False) -> str:
    """Build the host-check driver (which includes the runtime's API source)
    with the other sources, host parts instrumented by `kind` ("asan": address
    + undefined behaviour, "tsan": threads). Returns the executable's path."""
    san = SANITIZERS[kind]
    bdir = os.path.join(BUILD, "sanitize_" + kind)
    os.makedirs(bdir, exist_ok=True)
    driver = os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))
    srcs = [x for x in srcs if os.path.basename(x) != "sbqa_api.cpp"] + [driver]

    def comp(src):
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *COMMON, *san, "-Xarch_host", "-g"]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
        return obj

    with cf.ThreadPoolExecutor(min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    exe = os.path.join(bdir, "host_checks")
    cmd = [HIPCC, "--offload-arch=" + ARCH, *san, "-o", exe, *objs, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    if verbose:
        print("built", exe)
    return exe


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

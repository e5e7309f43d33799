"""Build libhank.so (gfx950) in-tree with hipcc.

    python -m paper_1501_01652_amd.build      # or: from paper_1501_01652_amd.build import build
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhank.so")
ARCH = os.environ.get("HANK_OFFLOAD_ARCH", "gfx950")

SOURCES = ["kernels.hip", "api.cpp", "planner.cpp", "tables.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(HERE, "..", "include")]
# packed FP32 instructions stay off (they are generated only when enabled)
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _compile(src: str, extra=(), tag: str = "") -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + (("_" + tag) if tag else "") + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [HIPCC] + COMMON + list(extra) + DEVICE + ["-c", path, "-o", obj]
    else:
        cmd = [HIPCC] + COMMON + list(extra) + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                                                "-x", "c++", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                     if "not a recognized feature" not in line)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s" % (" ".join(cmd), msgs))
    if msgs.strip():
        sys.stderr.write(msgs + "\n")
    return obj


def build(verbose: bool = True, lib: str = LIB, defines=()) -> str:
    """Compile every source and link `lib`; `defines` are extra -D flags."""
    os.makedirs(BUILD, exist_ok=True)
    extra = ["-D" + d for d in defines]
    tag = "_".join(d.replace("=", "") for d in defines)
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda s: _compile(s, extra, tag), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build()

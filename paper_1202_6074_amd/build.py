"""In-tree build of libcmlbm.so for gfx950 (hipcc), and of the host-only
build of the per-cell arithmetic used by the CPU tests."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcmlbm.so")
HOSTLIB = os.path.join(HERE, "libcmlbm_hostmath.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse multiply-adds only within an expression, as written: the default
    # (fuse across statements) decides per kernel, so that the same collision
    # could round differently in the step kernels of different schemes
    "-ffp-contract=on",
    "-Wl,-rpath,/opt/rocm/lib",
    "-I" + os.path.join(ROOT, "include"),
]
SOURCES = [os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "kernels2d.hip"), os.path.join(CSRC, "capi.cpp")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def build_hip(out=LIB):
    """Compile each source to an object in parallel, then link the shared library."""
    from concurrent.futures import ThreadPoolExecutor
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cflags = [f for f in HIP_FLAGS if f not in ("-shared",) and not f.startswith("-Wl,")]
    objs = [os.path.join(objdir, os.path.basename(src) + ".o") for src in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        list(ex.map(lambda so: _run([HIPCC] + cflags + ["-c", "-o", so[1], so[0]]), zip(SOURCES, objs)))
    tmp = out + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp] + objs)
    os.replace(tmp, out)
    return out


def build_hostmath(out=HOSTLIB):
    """Host (CPU) build of cm_math.hpp behind a small C interface, for tests."""
    src = os.path.join(CSRC, "hostmath.cpp")
    tmp = out + ".tmp"
    _run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, out)
    return out


def build():
    build_hip()
    build_hostmath()


if __name__ == "__main__":
    build()
    print("built", LIB, HOSTLIB)

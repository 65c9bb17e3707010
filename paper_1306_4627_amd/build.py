"""Build the gfx950 HIP library ``liblcs_hip.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblcs_hip.so")
SOURCES = ["prep.hip", "fill.hip", "halves.hip", "traceback.hip", "lcs_api.hip", "server.cpp",
           "plan.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# gfx950 only; packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build_library(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-Wall", "-I", CSRC, "-I", INCLUDE]
        if src.endswith(".hip"):
            cmd += ["-x", "hip"] + DEVICE_FLAGS
        cmd += ["-c", path, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        msg = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                        if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{msg}")
        if verbose and msg.strip():
            print(msg, file=sys.stderr)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC"] + DEVICE_FLAGS + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


STRIPED_SRC = os.path.join(HERE, "host", "striped.c")
STRIPED_LIB = os.path.join(HERE, "libstriped.so")


def build_striped() -> str:
    """The host baseline of the paper's row-striped OpenMP method."""
    tmp = STRIPED_LIB + ".tmp"
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall",
           "-o", tmp, STRIPED_SRC]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for striped.c:\n" + r.stdout + r.stderr)
    os.replace(tmp, STRIPED_LIB)
    return STRIPED_LIB


if __name__ == "__main__":
    print(build_library(verbose=True))
    print(build_striped())

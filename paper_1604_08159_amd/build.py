"""Build step of the gfx950 library, in-tree.

Produces ``libmra.so`` next to this file from ``csrc/*.hip``.  Every HIP
source is compiled for gfx950 only, with packed FP32 instructions disabled,
as its own translation unit (the sources share no device symbols), in
parallel, then linked into one shared library.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libmra.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
OBJDIR = os.path.join(HERE, "_build")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]


def hipcc() -> str:
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found: the gfx950 library cannot be built")
    return path


def _filtered(res: subprocess.CompletedProcess) -> list:
    return [l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l]


def build_library(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    cc = hipcc()

    def compile_one(src: str):
        obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
        res = subprocess.run([cc] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        return src, obj, res

    jobs = min(len(SOURCES), 8)
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, SOURCES))
    msgs = []
    for src, _, res in results:
        m = _filtered(res)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n" + "\n".join(m))
        msgs += m
    tmp = LIB + ".tmp"
    res = subprocess.run([cc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in results],
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + "\n".join(_filtered(res)))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose=True))

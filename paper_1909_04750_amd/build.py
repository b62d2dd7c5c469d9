"""Build libmickey.so (HIP, gfx950) in-tree with hipcc: every source compiled to an object
file in parallel, then linked into one shared library."""
from __future__ import annotations

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB_DIR = os.path.join(PKG, "lib")
OBJ_DIR = os.path.join(LIB_DIR, "obj")
LIB_PATH = os.path.join(LIB_DIR, "libmickey.so")
SOURCES = ["mickey_kernels.hip", "mickey_resume.hip", "mickey_batch.hip", "mickey_serve.hip", "grain_kernels.hip",
           "aes_kernels.hip", "mickey128_kernels.hip"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags() -> list:
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            # packed fp32 VALU forms are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(os.path.dirname(PKG), "include")]


def build_library(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every HIP source and link lib/libmickey.so (always recompiles)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc = hipcc()
    tag = "%d" % os.getpid()

    def compile_one(src: str) -> str:
        obj = os.path.join(OBJ_DIR, src.replace(".hip", ".%s.o" % tag))
        cmd = [cc] + compile_flags() + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed on %s:\n%s%s" % (src, res.stdout, res.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB_PATH + ".tmp" + tag
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    for o in objs:
        os.remove(o)
    if res.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build_library(verbose=True))

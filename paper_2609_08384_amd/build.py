"""Build the HIP engine library (libbrahms.so) in-tree for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libbrahms.so")

# the pass kernels of the heaviest line lengths first (the longest compiles),
# then the host logic
SOURCES = ["len_144.hip", "len_72.hip", "len_256.hip", "len_96.hip", "len_9_18.hip", "len_192.hip",
           "len_128.hip", "len_48_64.hip", "len_24_32.hip", "len_small.hip", "len_long.hip", "engine.hip",
           "adjoint.hip", "batch.hip", "diag.hip", "noalloc.hip"]
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # keep the compiler from emitting packed FP32 (v_pk_*_f32) instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the engine)")


def build(verbose: bool = False) -> str:
    """Compile every HIP source (in parallel) and link LIB (always recompiles)."""
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    procs, objs = [], []
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    for src in SOURCES:
        while sum(pr.poll() is None for _, pr in procs) >= jobs:
            import time
            time.sleep(0.2)
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc(), *compile_flags, "-c", "-I", os.path.join(ROOT, "include"),
               os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
        objs.append(obj)
    for cmd, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + out + err)
    tmp = LIB + ".tmp"
    link = [hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

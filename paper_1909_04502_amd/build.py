"""Build the HIP library ``librlbm.so`` for gfx950 in place (next to this file).

Run as ``python -m paper_1909_04502_amd.build`` or through ``__graft_entry__.build()``.
hipcc cross-compiles without a GPU.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/kernels.hip", "csrc/api.hip", "csrc/adjoint.hip", "csrc/batch.hip", "csrc/bandwidth.hip",
           "csrc/precompute.cpp", "csrc/massive.cpp"]
LIB = os.path.join(HERE, "librlbm.so")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep hipcc from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=HERE, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in res.stderr.splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError("build step failed:\n" + " ".join(cmd) + "\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object file under _build/ (in parallel, at most `jobs` at once;
    0 = one per source up to the CPU count), then link librlbm.so."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        path = os.path.join(HERE, src)
        if src.endswith(".hip"):
            cmd = [hipcc()] + FLAGS + ["-c", path, "-o", obj]
        else:   # host-only C++ (no device code)
            cmd = [hipcc(), "-O3", "-std=c++17", "-fPIC", "-x", "c++", "-D__HIP_PLATFORM_AMD__",
                   "-I/opt/rocm/include", "-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)
    workers = jobs if jobs > 0 else max(1, min(len(cmds), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        for fut in [ex.submit(_run, c, verbose) for c in cmds]:
            fut.result()
    tmp = LIB + ".tmp"
    _run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs, verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

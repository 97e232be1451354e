"""Compile the HIP library (gfx950) in-tree: paper_2606_07156_amd/libamp.so.

Device code and host code are compiled by hipcc; the shared library is then
linked against the HIP runtime that PyTorch bundles, so that a process which
also uses torch (for device memory and streams) holds one HIP/HSA runtime.
Set AMP_HIP_RUNTIME=system to link /opt/rocm's runtime instead.
"""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "scan_ph1.hip", "scan_ph2.hip", "scan_ph3.hip", "cl.hip", "noalloc.hip", "capi.cpp", "train.cpp", "build.cpp", "clmap.cpp", "server.cpp", "tune.cpp")]
OUT = os.path.join(HERE, "libamp.so")
BUILD = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
CFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-result",
    "-Wno-unused-value",
]


def _torch_lib_dir():
    import importlib.util

    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        return None
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    return d if glob.glob(os.path.join(d, "libamdhip64.so*")) else None


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError(f"build step failed: {cmd[0]}")
    if verbose and msgs:
        print("\n".join(msgs))


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs = [os.path.join(BUILD, os.path.basename(s) + ".o") for s in SRC]
    # the translation units compile concurrently (the kernels dominate)
    with concurrent.futures.ThreadPoolExecutor(len(SRC)) as pool:
        for f in [pool.submit(_run, [HIPCC, *CFLAGS, "-c", "-o", o, s], verbose) for s, o in zip(SRC, objs)]:
            f.result()
    tdir = None if os.environ.get("AMP_HIP_RUNTIME") == "system" else _torch_lib_dir()
    if tdir:
        rt = ["-L" + tdir, "-l:libamdhip64.so", "-Wl,-rpath," + tdir]
    else:
        rt = ["-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    _run(["g++", "-shared", "-o", OUT + ".tmp", *objs, *rt, "-Wl,--no-undefined", "-lstdc++", "-pthread"], verbose)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))

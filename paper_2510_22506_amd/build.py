"""Build libfctn.so (all HIP sources under csrc/) for gfx950 with hipcc.

Each source is compiled to its own object in parallel (every kernel is
launched from the file that defines it, so no relocatable device code is
needed), then the objects are linked into one shared library."""

import concurrent.futures
import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libfctn.so")
OBJ = os.path.join(ROOT, "_build")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)


def build(verbose=False):
    """Compile every csrc/*.hip file into paper_2510_22506_amd/libfctn.so."""
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = []
    for src in srcs:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append((obj, [hipcc, *HIPCC_FLAGS, *inc, "-c", src, "-o", obj]))
    if verbose:
        for _, cmd in jobs:
            print(" ".join(cmd), flush=True)
    workers = max(1, min(len(jobs), os.cpu_count() or 1, 8))
    with concurrent.futures.ThreadPoolExecutor(workers) as ex:
        list(ex.map(_run, [cmd for _, cmd in jobs]))
    tmp = LIB + ".tmp"
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc))), "lib")
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs],
          "-L", rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the in-tree shared library libwh2wav.so (HIP kernels for gfx950 + host planner).

The host planner (binary128 arithmetic, libquadmath) is compiled with g++;
the kernels and the C-ABI entry points with hipcc for gfx950.  Packed FP32
instructions are disabled for all device code.  The library is written next
to this file so that it travels with the source tree.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libwh2wav.so")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = "gfx950"
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-I", os.path.join(ROOT, "include"),
]
CXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-Wall", "-I", os.path.join(ROOT, "include")]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"build step failed: {' '.join(cmd[:3])} ...")
    return res


def build(verbose=False):
    """Compile every source and link libwh2wav.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for src in sorted(os.listdir(CSRC)):
        path = os.path.join(CSRC, src)
        base, ext = os.path.splitext(src)
        obj = os.path.join(BUILD, base + ".o")
        if ext == ".cpp":
            jobs.append(([shutil.which("g++") or "g++"] + CXX_FLAGS + ["-c", path, "-o", obj], obj))
        elif ext == ".hip":
            jobs.append(([HIPCC] + HIP_FLAGS + ["-c", path, "-o", obj], obj))
    # one compiler process per source file, side by side
    workers = max(1, min(len(jobs), int(os.environ.get("MAX_JOBS", "4"))))
    with concurrent.futures.ThreadPoolExecutor(workers) as pool:
        for f in [pool.submit(_run, cmd, verbose) for cmd, _ in jobs]:
            f.result()
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs + ["-lquadmath"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

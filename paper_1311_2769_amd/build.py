"""Build libhough.so (the HIP kernels and the C ABI) in-tree for gfx950.

Run as ``python -m paper_1311_2769_amd.build``.  Every build compiles from
source; nothing is cached outside the package directory.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libhough.so")
OBJ_DIR = os.path.join(ROOT, "_build", "libhough")
SOURCES = ["vote.hip", "peaks.hip", "vertex.hip", "assoc.hip", "api.hip", "noalloc.hip", "selftest.hip", "diag.hip",
           "tune.hip", "server.hip"]
ARCH = "gfx950"

# -ffp-contract=off: the vote arithmetic is specified op by op (no FMA).
# The default correctly rounded fp32 divide and denormal handling are kept.
# Packed fp32 instructions are disabled for all device code.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every uniform-address atomic here is already issued by one lane; the
    # atomic optimizer only wraps those in an extra wavefront reduction
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP library cannot be built")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhough.so")
    noise = [l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")


def build(verbose: bool = False, jobs: int = 0) -> str:
    """Compile every source to an object (in parallel) and link the library."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(OBJ_DIR, exist_ok=True)
    cc = hipcc()
    compile_flags = [f for f in FLAGS if f != "-shared"]
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[cc, *compile_flags, "-c", "-I", INCLUDE, "-I", CSRC, "-o", o, os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    jobs = jobs or min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as pool:
        list(pool.map(lambda c: _run(c, verbose), cmds))
    out_tmp = LIB + ".tmp"
    # the server marks its phases as roctx ranges (seen by rocprofv3 --marker-trace)
    _run([cc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out_tmp, *objs, "-L/opt/rocm/lib",
          "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"], verbose)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library ``libtilt.so`` in-tree for gfx950.

Usage: ``python paper_1205_5351_amd/build.py`` (run as a script so the
package, which loads the library, is not imported first).
The library is plain hipcc output: no PyTorch headers, no JIT cache.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
REPO_DIR = os.path.dirname(PKG_DIR)
CSRC = os.path.join(PKG_DIR, "csrc")
INCLUDE = os.path.join(REPO_DIR, "include")
LIB_NAME = "libtilt.so"
LIB_PATH = os.path.join(PKG_DIR, LIB_NAME)

SOURCES = ["tilt_kernels.hip", "tilt_peaks.hip", "tilt_noalloc.hip", "tilt_svdws.hip", "tilt_api.cpp",
           "tilt_serve.cpp", "tilt_rasl.cpp"]
ARCH = "gfx950"


def hipcc_path() -> str:
    p = shutil.which("hipcc")
    if p:
        return p
    cand = "/opt/rocm/bin/hipcc"
    if os.path.exists(cand):
        return cand
    raise RuntimeError("hipcc not found")


def compile_flags():
    return [
        f"--offload-arch={ARCH}",
        "-O3",
        "-std=c++17",
        "-fPIC",
        # packed FP32 instructions are disabled for all device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # no implicit multiply-add contraction: every fused multiply-add is
        # an explicit fmaf, so a device function gives the same bits in
        # every kernel it is inlined into (plain path == batched path)
        "-ffp-contract=off",
        f"-I{INCLUDE}",
        f"-I{CSRC}",
        "-Wno-unused-command-line-argument",
    ]


def build(verbose: bool = False) -> str:
    """Compile every source and link ``libtilt.so`` next to this file."""
    hipcc = hipcc_path()
    objs = []
    tmp = LIB_PATH + ".tmp"
    for src in SOURCES:
        srcp = os.path.join(CSRC, src)
        obj = os.path.join(PKG_DIR, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc] + compile_flags() + ["-c", srcp, "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc] + compile_flags() + ["-x", "hip", "-c", srcp, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        objs.append(obj)
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

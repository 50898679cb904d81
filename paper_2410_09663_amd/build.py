"""Build liboic.so (the HIP library behind include/oic.h) in-tree for gfx950.

Usage: python -m paper_2410_09663_amd.build   (or build() from Python).
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "liboic.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep the compiler from forming packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas", "-pthread",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")) +
                  glob.glob(os.path.join(PKG, "csrc", "*.cpp")))


def build(verbose: bool = False) -> str:
    """Compile every HIP source into liboic.so; always recompiles.  The sources compile
    to objects in parallel (each holds its own gfx950 code object), then link."""
    import shutil
    import tempfile

    tmpdir = tempfile.mkdtemp(prefix="oic_build_")
    try:
        compile_flags = [f for f in FLAGS if f != "-shared"]
        jobs = []
        for src in sources():
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            cmd = [HIPCC, *compile_flags, "-c", "-I", os.path.join(ROOT, "include"), "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append((obj, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                                               text=True)))
        failed = False
        for obj, proc in jobs:
            out, _ = proc.communicate()
            if proc.returncode != 0:
                sys.stderr.write(out)
                failed = True
        if failed:
            raise RuntimeError("hipcc failed building liboic.so")
        tmp = LIB + ".tmp"
        cmd = [HIPCC, *FLAGS, "-o", tmp, *[o for o, _ in jobs]]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking liboic.so")
        os.replace(tmp, LIB)
    finally:
        shutil.rmtree(tmpdir, ignore_errors=True)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

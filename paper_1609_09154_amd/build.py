"""Builds libnmf_mi355x.so (all HIP sources, gfx950) in the package folder.

Usage: python -m paper_1609_09154_amd.build   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SOURCES = ["gemm.hip", "gemm_bf16.hip", "update.hip", "objective.hip", "sparse.hip", "bpp.hip", "autograd.hip", "api.hip"]
LIB_NAME = "libnmf_mi355x.so"
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags():
    return [
        "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
        "-I" + os.path.join(ROOT, "include"),
        # packed FP32 instructions are kept out of every kernel
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # the row-local kernels rely on fully unrolled loops over the rank
        "-mllvm", "-pragma-unroll-threshold=1000000",
        "-Wno-unused-result",
    ]


def build(verbose: bool = False, jobs: int = 6) -> str:
    """Compile every source to an object in parallel, then link the library."""
    cc = hipcc()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [cc] + flags() + ["-c", os.path.join(HERE, "csrc", src), "-o", obj]
        procs.append((src, cmd))
    running = []
    failed = []
    for src, cmd in procs:
        while len(running) >= jobs:
            s, p = running.pop(0)
            out, _ = p.communicate()
            if p.returncode != 0:
                failed.append((s, out))
            elif verbose:
                sys.stdout.write(out.decode(errors="replace"))
        running.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for s, p in running:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append((s, out))
        elif verbose:
            sys.stdout.write(out.decode(errors="replace"))
    if failed:
        msg = "\n".join("%s:\n%s" % (s, o.decode(errors="replace")) for s, o in failed)
        raise RuntimeError("HIP compile failed\n" + msg)
    lib = os.path.join(HERE, LIB_NAME)
    tmp = lib + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))

"""Builds libtpf.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_2403_04578_amd.build          # compile what changed
    python -m paper_2403_04578_amd.build --force  # compile everything

Objects go to ``paper_2403_04578_amd/_build/``; the library lands next to this
file so that it travels with the source tree.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
REPO = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtpf.so")
ARCH = os.environ.get("TPF_OFFLOAD_ARCH", "gfx950")

SOURCES = ["network.cpp", "capi.cpp", "fpi_small.hip", "fpi_mixed.hip", "mismatch.hip", "mlp.hip", "fpi_large.hip",
           "fpi_tree.hip", "noalloc.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # MFMA accumulators stay in VGPRs (no AGPR copies around the k-loops)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-I", os.path.join(REPO, "include"),
]


def _headers_mtime() -> float:
    hs = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    hs.append(os.path.join(REPO, "include", "tpf.h"))
    return max(os.path.getmtime(h) for h in hs)


def _compile(src: str, force: bool, hmt: float) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    if not force and os.path.exists(obj) and os.path.getmtime(obj) >= max(os.path.getmtime(path), hmt):
        return obj
    cmd = ["hipcc", "-x", "hip", *FLAGS, "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-8000:]}")
    return obj


def build(force: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hmt = _headers_mtime()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, force, hmt), SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", *FLAGS, "-shared", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--force", action="store_true")
    ap.add_argument("-j", type=int, default=8)
    a = ap.parse_args()
    print(build(a.force, a.j))
    sys.exit(0)

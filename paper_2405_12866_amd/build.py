"""Build of the HIP library libqfs_hip.so for gfx950 (MI355X), in-tree.

Every HIP source is compiled by hipcc with packed-FP32 instruction selection
disabled; the shared library is written next to this file.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqfs_hip.so")
SOURCES = ["rng.hip", "linalg.hip", "sweep.hip", "group.hip", "engine.hip", "batch.hip",
           "batch_engine.hip", "mlp.hip", "learned.hip", "qudit.hip", "noalloc.hip"]
ARCH = os.environ.get("QFS_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
    "-Wno-unused-command-line-argument",
]


# Per-source flags. group.hip: common-code sinking off, so the switch over a gate's item
# slots keeps one body per case and the 16-element items stay in registers (merged cases
# select between array elements, which moves the items to scratch memory).
SOURCE_FLAGS = {"group.hip": ["-mllvm", "-simplifycfg-sink-common=false"]}


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source (always, even when a library exists) and link."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = ["hipcc", *FLAGS, *SOURCE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0))
    for p in procs:
        _wait(p)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", *FLAGS, "-shared", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _wait(item):
    src, p = item
    out, _ = p.communicate()
    text = out.decode(errors="replace")
    if p.returncode != 0:
        sys.stderr.write(text)
        raise RuntimeError(f"hipcc failed on {src}")
    warn = [ln for ln in text.splitlines() if "warning" in ln and "packed-fp32-ops" not in ln]
    if warn:
        sys.stderr.write("\n".join(warn) + "\n")


if __name__ == "__main__":
    print(build(verbose=True))

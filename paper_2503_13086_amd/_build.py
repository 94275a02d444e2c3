"""Build the HIP library (libgsmi.so) in-tree for gfx950 with hipcc.

Each source compiles to an object under _build/ (in parallel) and the objects link
into paper_2503_13086_amd/libgsmi.so.  Always recompiles: this is the build check.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgsmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["gs_api.hip", "k_preprocess.hip", "k_sort.hip", "k_raster.hip", "k_loss.hip", "k_adam.hip",
           "k_probe.hip", "gs_sched.hip"]

# Packed fp32 instructions are disabled for every HIP translation unit.
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-I", INCLUDE, "-I", CSRC]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stdout + r.stderr


# Per-source flags.  The raster kernels' LDS and global atomics take per-lane
# addresses by design; the compiler's wave-level atomic combining (which funnels an
# atomic through a read-lane loop when it can prove the address uniform) has
# nothing to gain there and is switched off for that file.
EXTRA = {"k_raster.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]}


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, *EXTRA.get(src, []), "-c", os.path.join(CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        outs = list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    outs.append(_run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]))
    os.replace(tmp, LIB)
    log = "\n".join(o for o in outs if o.strip())
    if verbose and log:
        print(log, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))

"""Build the HIP library ``libaxhosfem.so`` for gfx950 with hipcc (in-tree).

Each source under ``csrc/`` compiles to an object in ``_build/`` in parallel; the objects link
into ``paper_2504_07042_amd/libaxhosfem.so``.  Runs without a GPU (hipcc cross-compiles).

The same call builds the debug twin ``libaxhosfem_ldspoison.so``: the sources whose kernels use
LDS are compiled again with ``-DAX_LDS_POISON=1`` (every such kernel fills its LDS with NaN
before first use, so a read of an unwritten word shows up as NaN in the output) and linked with
the other objects of the normal build.  Select it with ``AXHOSFEM_LIB=<path>``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libaxhosfem.so")
LIB_POISON = os.path.join(PKG, "libaxhosfem_ldspoison.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are turned off for every HIP translation unit.
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(ROOT, "include")]

SOURCES = ["ax_common.cpp", "ax_local.hip", "ax_local_f64.hip", "ax_local_f32.hip", "ax_local_f16.hip",
           "item_f64.hip", "item_f32.hip", "ax_setup.hip", "gs.hip", "cg.hip", "batched.hip", "probe.hip"]
# sources whose kernels hold LDS arrays: recompiled for the poisoned debug twin
LDS_SOURCES = ["ax_local_f64.hip", "ax_local_f32.hip", "ax_local_f16.hip", "item_f64.hip", "item_f32.hip",
               "batched.hip"]


def _compile(job) -> str:
    src, variant = job
    path = os.path.join(CSRC, src)
    odir = os.path.join(BUILD, variant) if variant else BUILD
    os.makedirs(odir, exist_ok=True)
    obj = os.path.join(odir, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    extra = ["-DAX_LDS_POISON=1"] if variant == "ldspoison" else []
    cmd = [HIPCC] + FLAGS + extra + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} ({variant or 'release'}):\n{r.stderr}")
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False, jobs: int | None = None, poison: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    work = [(s, "") for s in SOURCES] + ([(s, "ldspoison") for s in LDS_SOURCES] if poison else [])
    # the longest translation units first, so the pool stays busy to the end
    work.sort(key=lambda j: j[0] not in LDS_SOURCES)
    jobs = jobs or min(len(work), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = dict(zip(work, ex.map(_compile, work)))
    _link([objs[(s, "")] for s in SOURCES], LIB)
    if verbose:
        print(f"built {LIB}")
    if poison:
        _link([objs[(s, "ldspoison")] if s in LDS_SOURCES else objs[(s, "")] for s in SOURCES], LIB_POISON)
        if verbose:
            print(f"built {LIB_POISON}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, poison="--no-poison" not in sys.argv)
    sys.exit(0)

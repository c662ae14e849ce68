"""Build ``libiga.so`` (the HIP C-ABI library) in-tree for gfx950.

Every translation unit is compiled with hipcc (device code for gfx950 only,
packed-FP32 instructions disabled) in parallel, then linked into
``paper_2604_19370_amd/libiga.so``.  ``python -m paper_2604_19370_amd.build``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libiga.so")
OBJ = os.path.join(HERE, "_build")
ROOT = os.path.dirname(HERE)

HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         f"-I{os.path.join(ROOT, 'include')}"]

SOURCES = ["plan.cpp", "api.cpp", "noalloc.cpp", "ensemble.cpp", "factor.hip", "assemble.hip", "sweep.hip",
           "sweep_f1.hip", "sweep_f2.hip", "sweep_f3.hip", "sweep_d1.hip", "sweep_d2.hip",
           "sweep_d3.hip", "sweep_col.hip", "sample.hip"]


def _compile(src: str) -> tuple[str, float, str]:
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    t0 = time.time()
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    log = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{log}")
    return obj, time.time() - t0, log


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, SOURCES))
    for (obj, dt, log), src in zip(results, SOURCES):
        if verbose:
            print(f"  {src}: {dt:.1f}s")
        if log.strip() and verbose:
            print(log)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp] + [r[0] for r in results]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} in {time.time() - t0:.1f}s")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Compile libensdns.so (HIP C++ for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["csrc/ens_api.cpp", "csrc/kernels_step.hip", "csrc/kernels_misc.hip", "csrc/kernels_stats.hip",
           "csrc/kernels_diag.hip", "csrc/kernels_lambda.hip"]
HEADERS = ["csrc/ens_internal.h", "csrc/ens_diag.h", "csrc/ens_lambda.h", "csrc/fft.hpp", "csrc/gmem.hpp", "../include/ens.h"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-fvisibility=hidden",
         "-Wno-unused-result", "-Wno-unused-value",
         # no packed-FP32 instructions: hipcc would otherwise form them from scalar float code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
LIB = os.path.join(HERE, "libensdns.so")


def _compile(src: str, obj: str) -> None:
    cmd = ["hipcc", *FLAGS, "-c", os.path.join(HERE, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")


def build(jobs: int = 4) -> str:
    """Compile every source (always) and link libensdns.so; returns its path."""
    out = os.path.join(HERE, "_build")
    os.makedirs(out, exist_ok=True)
    objs = [os.path.join(out, os.path.basename(s) + ".o") for s in SOURCES]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(lambda so: _compile(*so), zip(SOURCES, objs)))
    tmp = LIB + ".tmp"
    r = subprocess.run(["hipcc", "-shared", "--offload-arch=gfx950", "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())

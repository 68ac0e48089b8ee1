"""Compiles the gfx950 libraries in-tree with hipcc.

    libringo.so      the conversion library (C ABI declared in include/ringo.h)
    libringo_gen.so  the seeded workload generators (host and device)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("RINGO_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]

LIBS = {
    "libringo.so": ["kernels.hip", "lsd_d8.hip", "lsd_d9.hip", "lsd_d10.hip", "lsd_d11.hip", "hash.hip",
                    "to_table.hip", "pagerank.hip", "small.hip", "pipeline.hip", "serve.hip"],
    "libringo_gen.so": ["workloads.hip"],
}


def _compile(src: str) -> str:
    os.makedirs(OBJ, exist_ok=True)
    obj = os.path.join(OBJ, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> list[str]:
    srcs = sorted({s for v in LIBS.values() for s in v if os.path.exists(os.path.join(CSRC, s))})
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = dict(zip(srcs, ex.map(_compile, srcs)))
    out = []
    for lib, parts in LIBS.items():
        parts = [objs[p] for p in parts if p in objs]
        target = os.path.join(HERE, lib)
        tmp = target + ".tmp"
        # -z defs: a symbol left undefined fails the link, not the first load
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-z,defs", "-o", tmp, *parts,
               "-lpthread"]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"link failed for {lib}:\n{r.stdout}\n{r.stderr}")
        os.replace(tmp, target)
        out.append(target)
        if verbose:
            print("built", target)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Build libcoffee.so (HIP for gfx950) in-tree.

Every `.hip` source under csrc/ is compiled with hipcc for gfx950, the pure
host `.cpp` sources with g++, all in parallel, and linked into
paper_1407_0904_amd/libcoffee.so. Objects go to _build/ at the repo root.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libcoffee.so")
BUILD = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-result", "-Wno-unknown-warning-option"]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall"]


def _sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(job):
    cmd, obj = job
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = _sources()
    work = []
    for f in hip:
        obj = os.path.join(BUILD, f + ".o")
        work.append(([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj], obj))
    for f in cpp:
        obj = os.path.join(BUILD, f + ".o")
        work.append((["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj], obj))
    jobs = jobs or min(8, os.cpu_count() or 4)
    # the heaviest translation units first
    work.sort(key=lambda w: -os.path.getsize(w[0][-3]))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, work))
    tmp = OUT + ".tmp"
    link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(link, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

"""Compiles libesg.so in-tree: HIP kernels + runtime for gfx950 (hipcc) and
the host index builder (g++ with OpenMP).  Objects go to _build/ at the
repository root; the library lands next to this file."""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libesg.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-ffp-contract=off",                     # distances: no contraction of x-q into fma
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-result",
]
CXX_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-fopenmp", "-march=x86-64-v3", "-Wall",
             "-ffp-contract=off"]


def dims() -> list[int]:
    only = os.environ.get("ESG_DIMS_ONLY")
    if only:
        return [int(only)]
    txt = open(os.path.join(CSRC, "esg_dims.h")).read()
    m = re.search(r"#define ESG_DIMS\(X\) X\(32\)(.*)", txt)
    return [32] + [int(v) for v in re.findall(r"X\((\d+)\)", m.group(1))]


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError(f"command failed: {' '.join(cmd)}\n{p.stdout}\n{p.stderr}")
    return p


def _newer(out: str, deps: list[str]) -> bool:
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(d) > t for d in deps)


def build(force: bool = False, jobs: int | None = None, verbose: bool = False) -> str:
    """Builds every kernel class; ESG_DIMS_ONLY=<d> (development only) builds
    the kernels of one class into _build/only<d>/ and the library with it."""
    global BUILD
    only = os.environ.get("ESG_DIMS_ONLY")
    if only:
        BUILD = os.path.join(ROOT, "_build", f"only{int(only)}")
        HIP_FLAGS.append(f"-DESG_DIMS_ONLY={int(only)}")
    os.makedirs(BUILD, exist_ok=True)
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers.append(os.path.join(ROOT, "include", "esg.h"))
    jobs = jobs or min(8, os.cpu_count() or 4)
    tasks = []
    objs = []
    inst = os.path.join(CSRC, "esg_search_inst.hip")
    for d in dims():
        o = os.path.join(BUILD, f"esg_search_d{d}.o")
        objs.append(o)
        if force or _newer(o, [inst] + headers):
            tasks.append([HIPCC, *HIP_FLAGS, f"-DESG_DIM={d}", "-c", inst, "-o", o])
    for src in sorted(os.listdir(CSRC)):
        if src.endswith(".hip") and src != "esg_search_inst.hip":
            o = os.path.join(BUILD, src[:-4] + ".o")
            objs.append(o)
            if force or _newer(o, [os.path.join(CSRC, src)] + headers):
                tasks.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
        elif src.endswith(".cpp"):
            o = os.path.join(BUILD, src[:-4] + ".o")
            objs.append(o)
            if force or _newer(o, [os.path.join(CSRC, src)] + headers):
                tasks.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, src), "-o", o])
    with cf.ThreadPoolExecutor(jobs) as ex:
        for cmd, _ in zip(tasks, ex.map(_run, tasks)):
            if verbose:
                print("built", cmd[-1], file=sys.stderr)
    # relink whenever the object set differs from the last link (a
    # single-class development build and the full build share LIB)
    stamp = os.path.join(ROOT, "_build", "libesg.objects")
    last = open(stamp).read() if os.path.exists(stamp) else ""
    if force or tasks or _newer(LIB, objs) or last != "\n".join(objs):
        tmp = LIB + ".tmp"
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs,
              "-lgomp", "-Wl,-z,defs"])
        os.replace(tmp, LIB)
        with open(stamp, "w") as f:
            f.write("\n".join(objs))
    return LIB


if __name__ == "__main__":
    build(force="--force" in sys.argv, verbose=True)
    print(LIB)

"""Build librmrt.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Usage: python -m paper_2206_00366_amd.build [-j JOBS]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librmrt.so")
# The checked library: the same code with every neighbour node index tested
# against the domain (RMRT_CHECKED = 1) in the FP64 kernels of every lattice
# and in the host code; the FP32 / FP16 kernels, whose index code is the same
# templates, are the production objects.
CHECKED_LIB = os.path.join(HERE, "librmrt_checked.so")
CHECKED_BUILD = os.path.join(BUILD, "checked")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# packed FP32 instructions are kept out of every kernel (-packed-fp32-ops)
FLAGS = ["-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include")]


def sources():
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    srcs += ["rmrt_capi.cpp", "nn_capi.cpp"]
    return [os.path.join(CSRC, s) for s in srcs]


def checked_unit(src: str) -> bool:
    name = os.path.basename(src)
    return name.endswith("_f64.hip") or name == "rmrt_capi.cpp"


def compile_one(src: str, checked: bool = False) -> str:
    out_dir = CHECKED_BUILD if checked else BUILD
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *FLAGS, *(["-DRMRT_CHECKED=1"] if checked else []), "-x", "hip", "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-4000:]}")
    return obj


def link(objs, lib: str) -> None:
    tmp = lib + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, lib)


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(CHECKED_BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 4)))
    checked_srcs = [s for s in srcs if checked_unit(s)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(compile_one, s) for s in srcs]
        cfuts = [ex.submit(compile_one, s, True) for s in checked_srcs]
        objs = [f.result() for f in futs]
        cobjs = {os.path.basename(s): f.result() for s, f in zip(checked_srcs, cfuts)}
    link(objs, LIB)
    if verbose:
        print(f"built {LIB}")
    link([cobjs.get(os.path.basename(s), o) for s, o in zip(srcs, objs)], CHECKED_LIB)
    if verbose:
        print(f"built {CHECKED_LIB}")
    build_examples(verbose)
    return LIB


EXAMPLES = os.path.join(HERE, "examples")


def build_examples(verbose: bool = True) -> None:
    """Plain-C programs that use the C ABI of librmrt.so (host code, gcc)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    for src in sorted(f for f in os.listdir(EXAMPLES) if f.endswith(".c")):
        exe = os.path.join(EXAMPLES, src[:-2])
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
               "-I", os.path.join(HERE, "..", "include"), "-I", os.path.join(rocm, "include"),
               os.path.join(EXAMPLES, src), "-o", exe, "-L", HERE, "-lrmrt",
               "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
               "-Wl,-rpath,$ORIGIN/..", "-Wl,-rpath," + os.path.join(rocm, "lib")]
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"gcc failed for {src}:\n{res.stderr[-4000:]}")
        if verbose:
            print(f"built {exe}")


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    a = ap.parse_args()
    try:
        build(a.j)
    except RuntimeError as e:
        print(e, file=sys.stderr)
        sys.exit(1)

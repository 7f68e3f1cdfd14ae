"""Build libmdseries.so (HIP, gfx950) in-tree.

Every .hip file under csrc/ is compiled separately with hipcc and the
objects are linked into paper_2012_06607_amd/libmdseries.so.  FP contraction
is off so that every multiple-double operation keeps its exact sequence of
roundings; packed FP32 instructions are disabled.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import re
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmdseries.so")
ARCH = os.environ.get("MDSERIES_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-fast-math", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


# Device functions allowed to stay real calls: leaf routines without LDS
# variables of their own (the series product of the five-limb and wider
# kernels).  Everything else must be inlined into its kernel: a call into a
# large function has shown two hazards here, long jumps that go through
# s[30:31] (the return address) and wrong results from a non-inlined
# function that declares LDS variables.
CALLABLE = (re.compile(r"^_ZN3mds15conv_block_call"),)


def check_device_asm(asm_path: str) -> list[str]:
    """Non-kernel device functions that were not inlined and are not on the
    CALLABLE list, or that jump through s[30:31].  Returns their symbols."""
    text = open(asm_path).read()
    kernels = set(re.findall(r"\.name:\s+(\S+)", text))
    functions = set(re.findall(r"\.type\s+(\S+),@function", text))
    labels = [(mm.start(), mm.group(1)) for mm in re.finditer(r"^(_Z\w+):", text, re.M)]
    bad = []
    for i, (pos, name) in enumerate(labels):
        if name in kernels or name not in functions:
            continue  # kernels, and data (device variables) rather than code
        end = labels[i + 1][0] if i + 1 < len(labels) else len(text)
        if "s_getpc_b64 s[30:31]" in text[pos:end] or not any(c.match(name) for c in CALLABLE):
            bad.append(name)
    return bad


def _compile(src: str) -> str:
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    cmd = [HIPCC, *FLAGS, "-save-temps=obj", "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=OBJ)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if os.environ.get("MDSERIES_BUILD_VERBOSE"):
        print(f"  {os.path.basename(src)}: {time.time() - t0:.0f} s", flush=True)
    asm = os.path.join(OBJ, os.path.basename(src)[:-4] + f"-hip-amdgcn-amd-amdhsa-{ARCH}.s")
    bad = check_device_asm(asm)
    if bad:
        raise RuntimeError(f"{src}: device functions left as calls (force-inline them): {bad}")
    return obj


def _includes(path: str, seen: set[str]) -> set[str]:
    """Files reached from `path` through #include "..." (quoted includes
    resolved next to the including file or in include/)."""
    for name in re.findall(r'^\s*#include\s+"([^"]+)"', open(path).read(), re.M):
        for base in (os.path.dirname(path), os.path.join(ROOT, "include")):
            cand = os.path.normpath(os.path.join(base, name))
            if os.path.exists(cand):
                if cand not in seen:
                    seen.add(cand)
                    _includes(cand, seen)
                break
    return seen


def _stale(src: str) -> bool:
    obj = os.path.join(OBJ, os.path.basename(src)[:-4] + ".o")
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(t < os.path.getmtime(f) for f in {src} | _includes(src, set()))


def build(jobs: int | None = None, verbose: bool = False, changed_only: bool = False) -> str:
    """Compile every kernel source and link the shared library; returns its
    path.  changed_only: recompile only the sources newer than their object
    (any header change recompiles everything)."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    todo = srcs
    if changed_only:
        todo = [s for s in srcs if _stale(s)]
    jobs = jobs or min(max(len(todo), 1), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, os.path.basename(s)[:-4] + ".o") for s in srcs]
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True, changed_only="--changed" in sys.argv)
    sys.exit(0)

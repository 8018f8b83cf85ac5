"""Builds libmm.so (the gfx950 kernels and the C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmm.so")
HOSTCOPY = os.path.join(PKG, "hostcopy")
HOSTCOPY_LIB = os.path.join(PKG, "libmm_hostcopy.so")
COBOUND_SRC = os.path.join(PKG, "cobound", "mm_cobound.hip")
COBOUND_EXE = os.path.join(PKG, "mm_cobound")
ARCH = "gfx950"
HIPFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    # binary32 results must match the CPU definition bit for bit: no
    # contraction; hipcc's default correctly rounded f32 divide stays on
    "-ffp-contract=off",
    # no packed-fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def hipcc() -> str:
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _spilling_kernels(remarks: str) -> list[str]:
    """Kernels whose resource-usage remark reports per-lane scratch (register
    spills or stack). The kernels are written to need none; a spill in a
    1024-thread kernel is also a sign that its register budget is exceeded."""
    bad, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            continue
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            bad.append(f"{name} ({m.group(1)} B/lane)")
    return bad


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(OUT, os.path.basename(src)[:-4] + ".o")
    cmd = [hipcc(), *HIPFLAGS, "-Rpass-analysis=kernel-resource-usage", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    bad = _spilling_kernels(r.stderr)
    if bad:
        raise RuntimeError(f"{os.path.basename(src)}: kernels use scratch: " + ", ".join(bad))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(len(srcs), max(1, (os.cpu_count() or 2) // 2))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    # -z defs: every symbol the library uses must resolve at link time
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Wl,-z,defs", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("linking libmm.so failed")
    os.replace(tmp, LIB)
    build_hostcopy()
    build_cobound()
    return LIB


def build_cobound() -> str:
    """The ALU co-bound microbenchmark of the bin pass (an executable; the
    bench runs it as a child process)."""
    tmp = COBOUND_EXE + ".tmp"
    cmd = [hipcc(), *HIPFLAGS, COBOUND_SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("building mm_cobound failed")
    os.replace(tmp, COBOUND_EXE)
    return COBOUND_EXE


def build_hostcopy() -> str:
    """The host-copy comparison renderer: plain C with OpenMP, binary32 with
    no contraction (its frames must equal the device path's)."""
    tmp = HOSTCOPY_LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-I", HOSTCOPY, os.path.join(HOSTCOPY, "hostcopy.c"),
           "-o", tmp, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("building libmm_hostcopy.so failed")
    os.replace(tmp, HOSTCOPY_LIB)
    return HOSTCOPY_LIB


if __name__ == "__main__":
    print(build(verbose=True))

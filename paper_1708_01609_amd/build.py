"""Build libbfsearch.so (gfx950) in-tree with hipcc.

Usage: python -m paper_1708_01609_amd.build  [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbfsearch.so")
# the runtime, the device tail sort, and the kernel sets of each storage precision (separate
# sources, so the template instantiations compile in parallel)
SOURCES = [os.path.join(CSRC, f) for f in ("bfsearch.hip", "bfs_tail_sort.hip", "bfs_ks_f32.hip", "bfs_ks_w16f.hip",
                                           "bfs_ks_w16b.hip", "bfs_ks_f64.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("bfs_device.h", "bfs_fft3.h", "bfs_kernels.h", "bfs_fused.h",
                                           "bfs_kernelset.h", "bfs_records.h", "bfs_runtime_kernels.h",
                                           "bfs_tail_sort.h")] + [
    os.path.join(ROOT, "include", "bfsearch.h")
]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # multiply-adds fused only within one source expression, so every
    # kernel instantiation (dense, threshold, projection) rounds alike
    "-ffp-contract=on",
    # packed FP32 VALU forms are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]
OBJDIR = os.path.join(HERE, "_build")


def compile_commands() -> list[list[str]]:
    """One hipcc -c per source (they compile in parallel), objects under _build/."""
    return [[hipcc(), *FLAGS, "-c", "-o", os.path.join(OBJDIR, os.path.basename(src) + ".o"), src]
            for src in SOURCES]


def link_command(out: str = LIB) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", out,
            *[os.path.join(OBJDIR, os.path.basename(src) + ".o") for src in SOURCES]]


def build(verbose: bool = False) -> str:
    """Compile the library (always; this is the build check) and return its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    cmds = compile_commands()
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    procs = [subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True) for c in cmds]
    failed = []
    for c, pr in zip(cmds, procs):
        out, _ = pr.communicate()
        if pr.returncode != 0:
            failed.append((c, pr.returncode, out))
    if failed:
        for c, rc, out in failed:
            sys.stderr.write(" ".join(c) + "\n" + out)
        raise RuntimeError(f"hipcc failed with exit code {failed[0][1]}")
    tmp = LIB + ".tmp"
    cmd = link_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc link failed with exit code {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))

"""Build ``libccg.so`` (the HIP kernels and the C ABI of include/ccg.h) for
gfx950 with hipcc, in-tree under ``paper_1208_4869_amd/_lib``."""
from __future__ import annotations

import os
import re
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libccg.so")
SOURCES = ["ccg_solvers.hip", "ccg_block.hip", "ccg_small.hip"]
HEADERS = ["ccg_device.h", "ccg_gemv.h", "ccg_krylov.h", "ccg_host.h", "ccg_t3.h"]
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"),
                 "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def scratch_kernels(remarks: str) -> list:
    """Kernels whose per-lane scratch (stack or spills) is not zero, from the
    compiler's kernel-resource-usage remarks."""
    found, name = [], None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and int(m.group(1)) > 0:
            found.append((name, int(m.group(1))))
    return found


def build(verbose: bool = False) -> str:
    """Compile every HIP source into LIB (always recompiles).  Fails when a
    kernel uses scratch memory: a stack object or a spill in a hot kernel
    costs far more than the registers it saves."""
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *FLAGS, "-Rpass-analysis=kernel-resource-usage",
           "-I", os.path.join(os.path.dirname(PKG), "include"),
           *[os.path.join(CSRC, s) for s in SOURCES], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(
            ln for ln in proc.stderr.splitlines() if "remark" not in ln))
    notes = [ln for ln in proc.stderr.splitlines()
             if ("warning:" in ln or "error" in ln) and "packed-fp32-ops" not in ln]
    if verbose and notes:
        print("\n".join(notes), flush=True)
    bad = scratch_kernels(proc.stderr)
    if bad:
        os.remove(tmp)
        raise RuntimeError("kernels using scratch memory: %s" % bad)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

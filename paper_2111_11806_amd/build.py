"""Build librbdi (HIP, gfx950) in-tree with hipcc.

The library is compiled from ``csrc/rbdi_api.hip`` (which includes the
kernel and physics headers) into ``paper_2111_11806_amd/_lib/librbdi.so``.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "librbdi.so")
SOURCES = ["rbdi_api.hip"]
HEADERS = ["rbdi_batch.hpp", "rbdi_kernels.hpp", "rbdi_mlp.hpp", "rbdi_physics.hpp"]
ARCH = os.environ.get("RBDI_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    # keep packed-FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # Kernels take the launch parameters (a ~2 KB struct) by value and read
    # them through references. Clang copies such an argument into a private
    # stack slot, which InstCombine folds back into reads of the kernel
    # argument only while the slot has at most 300 users (its default); the
    # sweeps with the most inlined physics exceed that, and the copy then
    # lands in scratch memory (2 KB per lane).
    "-mllvm", "-instcombine-max-copied-from-constant-users=4000",
    # No machine-level loop-invariant code motion. A VALU instruction reads at
    # most one scalar operand, so the sweeps move many material and grid
    # constants into vector registers; inside the tile sweeps' column loop
    # that pass hoists those moves out of the loop and keeps them live across
    # it: the FP32 elastoplastic tile sweeps then spilled 31-47 registers at
    # 256 VGPRs, and with the moves left at their uses they take 237, no spill.
    "-mllvm", "-disable-machine-licm",
]


def hipcc():
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def build(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always when force, else only if missing/stale)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(HERE, "..", "include", "rbdi.h")]
    if not force and os.path.exists(LIB):
        t = os.path.getmtime(LIB)
        if all(os.path.getmtime(d) <= t for d in deps):
            return LIB
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-o", tmp] + srcs
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))

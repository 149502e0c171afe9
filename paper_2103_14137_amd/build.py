"""Build the HIP library libuvc.so in-tree for gfx950 with hipcc.

    python -m paper_2103_14137_amd.build

Every .hip file under csrc/ is compiled into one shared library next to this
file.  The build always recompiles (it is the "does it build" check).
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libuvc.so")
ARCH = os.environ.get("UVC_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    "-Wno-unused-command-line-argument",
    # Packed FP32 (v_pk_*_f32) stays off: the FP32 fast path is written as
    # scalar FP32 arithmetic and must compile to scalar FP32 instructions.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    f"-I{os.path.join(ROOT, 'include')}",
]


def hipcc() -> str:
    p = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(p):
        raise RuntimeError("hipcc not found")
    return p


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_asm(out_dir: str) -> None:
    """Write the gfx950 assembly of every source (for inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    for src in sources():
        if not src.endswith(".hip"):
            continue
        base = os.path.splitext(os.path.basename(src))[0]
        cmd = [hipcc(), *[f for f in HIPCC_FLAGS if f not in ("-shared", "-fPIC")], "--cuda-device-only", "-S",
               src, "-o", os.path.join(out_dir, base + ".s")]
        subprocess.check_call(cmd)


if __name__ == "__main__":
    build(verbose=True)
    if len(sys.argv) > 1 and sys.argv[1] == "--asm":
        build_asm(sys.argv[2] if len(sys.argv) > 2 else os.path.join(ROOT, "_build", "asm"))
    print(LIB)

"""Builds libga.so (HIP, gfx950) in-tree with hipcc."""

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libga.so")
SRCS = [os.path.join(PKG, "csrc", f) for f in ("ga_lib.hip", "ga_server.hip", "ga_batch.hip")]
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3",
    "-std=c++20",
    f"--offload-arch={ARCH}",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
]


def sources():
    csrc = os.path.join(PKG, "csrc")
    return sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith((".hip", ".hpp", ".h")))


def build_lib(verbose: bool = False) -> str:
    """Compile csrc/ga_lib.hip, csrc/ga_server.hip and csrc/ga_batch.hip into
    paper_1711_05017_amd/libga.so (always recompiles). Returns the library
    path."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I", os.path.join(ROOT, "include"), "-o", tmp, *SRCS, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_lib(verbose=False))

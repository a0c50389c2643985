"""Build libpanda.so for gfx950 with hipcc (in-tree, next to this file)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpanda.so")
SOURCES = ["panda_api.hip", "batch_api.hip", "warm_api.hip", "tanimoto_gemm.hip", "packed.hip",
           "update_kernels.hip", "batched.hip", "warmstart.hip", "null.hip"]

# Packed FP32 instructions are switched off for all device code; hipcc's host
# pass warns that it does not know the feature, which is harmless.
HIPFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument"]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the
# library (a CPU check of the host code: argument checks, layouts, the ABI);
# the device code is built as usual.  Loaded by the sanitizer test only.
LIB_SAN = os.path.join(HERE, "libpanda_san.so")
SANFLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
            "-shared-libsan"]


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    tmp = out + ".tmp%d" % os.getpid()
    cmd = (["/opt/rocm/bin/hipcc"] + HIPFLAGS + (SANFLAGS if sanitize else [])
           + ["-I", os.path.join(ROOT, "include"), "-o", tmp]
           + [os.path.join(CSRC, s) for s in SOURCES])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libpanda.so")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))

"""Compile the HIP library (libchromo_lbm.so) for gfx950 in-tree."""
import os
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libchromo_lbm.so")
SOURCES = [os.path.join(PKG, "csrc", "chromo_api.hip")]
HEADERS = [os.path.join(PKG, "csrc", "chromo_kernels.hpp"), os.path.join(ROOT, "include", "chromo_lbm.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed-FP32 VALU instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; install ROCm or put hipcc on PATH")
    return exe


def build(verbose=True):
    """Compile every source into the shared library (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I" + os.path.join(ROOT, "include"), "-o", tmp] + SOURCES
    t0 = time.time()
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s\n%s" % (res.returncode, " ".join(cmd), err))
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1f s" % (os.path.relpath(LIB, ROOT), time.time() - t0), flush=True)
        if err.strip():
            print(err, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

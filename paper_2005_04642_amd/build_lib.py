"""Compile the HIP library (libchromo_lbm.so) for gfx950 in-tree.

One translation unit per population storage format (their kernels are
independent template instantiations) plus the C ABI; the units compile in
parallel and are linked into one shared library."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import tempfile
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libchromo_lbm.so")
CSRC = os.path.join(PKG, "csrc")
SOURCES = [os.path.join(CSRC, f) for f in
           ("chromo_api.hip", "chromo_f32.hip", "chromo_f64.hip", "chromo_f16o.hip", "chromo_bf16o.hip")]
HEADERS = [os.path.join(CSRC, f) for f in ("chromo_kernels.hpp", "chromo_host.hpp", "chromo_launch.hpp",
                                           "chromo_adjoint.hpp")] + \
          [os.path.join(ROOT, "include", "chromo_lbm.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # multiply-add fusion only within one source expression: a site's arithmetic
    # is then the same in every unrolled copy of the march, so results do not
    # depend on how a lattice is cut into tiles
    "-ffp-contract=on",
    # no packed-FP32 VALU instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; install ROCm or put hipcc on PATH")
    return exe


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed (%d):\n%s\n%s" % (res.returncode, " ".join(cmd), err))
    return err


def build(verbose=True):
    """Compile every source into the shared library (always recompiles)."""
    t0 = time.time()
    inc = "-I" + os.path.join(ROOT, "include")
    with tempfile.TemporaryDirectory(prefix="chromo_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(s) + ".o") for s in SOURCES]
        jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with cf.ThreadPoolExecutor(jobs) as ex:
            errs = list(ex.map(lambda so: _run([hipcc()] + HIPCC_FLAGS + [inc, "-c", so[0], "-o", so[1]]),
                               zip(SOURCES, objs)))
        tmp = LIB + ".tmp"
        errs.append(_run([hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs))
    os.replace(tmp, LIB)
    if verbose:
        print("built %s in %.1f s" % (os.path.relpath(LIB, ROOT), time.time() - t0), flush=True)
        err = "\n".join(e for e in errs if e.strip())
        if err.strip():
            print(err, file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()

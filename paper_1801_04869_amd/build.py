"""Build the HIP library libmagfft.so for gfx950 (in-tree, next to this file).

Run as ``python -m paper_1801_04869_amd.build`` or call ``build()``.  Every
source under csrc/ is compiled with hipcc; packed-FP32 instructions are
disabled (-packed-fp32-ops) and the objects are linked into one shared
library exporting the C ABI of include/magfft.h.  The transform kernels
(film.hip, bulk.hip) let the compiler fuse multiplies and adds into FMAs; the
step controller (capi.hip) keeps every product and sum separately rounded, so
that its accept/reject decisions follow the same arithmetic as a plain
evaluation of the formulas.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libmagfft.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
         "-Wno-unused-result", "-Wno-unknown-pragmas"]

SOURCES = ["capi.hip", "film.hip", "bulk.hip", "noalloc.hip"]
CONTRACT = {"capi.hip": "-ffp-contract=off", "film.hip": "-ffp-contract=fast", "bulk.hip": "-ffp-contract=fast",
            "noalloc.hip": "-ffp-contract=off"}


def _compile(src):
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + [CONTRACT[src], "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-6000:]))
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)

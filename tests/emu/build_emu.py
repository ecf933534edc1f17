"""Build the CPU emulation of the HIP library (host C++ + AddressSanitizer).

TEST INFRASTRUCTURE ONLY.  The unmodified library sources are compiled as
host C++ against tests/emu/hip/hip_runtime.h, which runs every work-group on
CPU threads.  Used to bounds-check kernels and launch shapes on the CPU."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1801_04869_amd", "csrc")
OUT = os.path.join(HERE, "_build", "libmagfft_emu.so")


def build(asan=True):
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in ("capi.hip", "film.hip", "bulk.hip", "noalloc.hip")]
    newest = max(os.path.getmtime(p) for p in srcs + [os.path.join(HERE, "hip", "hip_runtime.h")] +
                 [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")])
    if os.path.exists(OUT) and os.path.getmtime(OUT) > newest:
        return OUT
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-I", HERE,
           "-DMAG_BULK_ENABLE=1", "-Wno-ignored-attributes", "-Wno-attributes", "-fno-omit-frame-pointer"]
    if asan:
        cmd += ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]
    cmd += ["-x", "c++"] + srcs + ["-o", OUT]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-8000:])
    return OUT


if __name__ == "__main__":
    print(build())

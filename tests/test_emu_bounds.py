"""CPU bounds check of the HIP sources: the library is compiled as host C++
with AddressSanitizer and UndefinedBehaviorSanitizer against a small emulation
of the HIP runtime (one CPU thread per work-item, real barriers, device memory
as a separate, poisoned address space, kernel pointer arguments and copy
kinds checked against the allocation registry), then run on small film and
bulk cases and compared with the FP64 oracle.  The launch shapes it records
are then checked against the gfx950 code objects of the same sources
(work-items per group within the compiled bound, static plus dynamic LDS
within the per-group limit).

The 3D path runs only here: it is held off the GPU (see the note in
capi.hip), and the emulation build alone enables it.  "bulk32" is the first
bulk case of the GPU parity tests (32^3 cube in a 32^3 grid, FP64, one inner
iteration)."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _libasan():
    r = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if p and os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("MAG_EMU") != "1",
                    reason="emulated-kernel runs take 5-15 min per case; MAG_EMU=1 runs them")
@pytest.mark.parametrize("which", ["film", "spectral", "radix3", "capture", "bulk", "bulk32"])
def test_emulated_kernels_in_bounds_and_match_oracle(which, tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    asan = _libasan()
    if asan is None:
        pytest.skip("libasan not found")
    sys.path.insert(0, ROOT)
    from tests.emu import build_emu
    lib = build_emu.build(asan=True)
    log = str(tmp_path / "launches.log")
    env = dict(os.environ)
    env["LD_PRELOAD"] = asan
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["EMU_LAUNCH_LOG"] = log
    r = subprocess.run([sys.executable, os.path.join(HERE, "emu", "emu_driver.py"), lib, which],
                       capture_output=True, text=True, env=env, cwd=ROOT, timeout=1800)
    print(r.stdout[-4000:])
    print(r.stderr[-4000:])
    assert r.returncode == 0
    assert "EMU_DONE fails=0" in r.stdout
    if shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
        return
    from tests.emu import kernel_limits
    seen, problems = kernel_limits.check(lib, log, os.path.join(ROOT, "paper_1801_04869_amd", "csrc"),
                                         ["capi.hip", "film.hip", "bulk.hip", "noalloc.hip"])
    assert seen
    assert not problems, problems

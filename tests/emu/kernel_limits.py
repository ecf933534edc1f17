"""Launch shapes of the CPU emulation against the gfx950 code objects.

TEST INFRASTRUCTURE ONLY.  The emulated library logs every launch (kernel
address relative to its shared object, grid, block, dynamic LDS bytes; see
tests/emu/hip/hip_runtime.h).  This module compiles the same sources for
gfx950 to device assembly with hipcc, reads each kernel's code-object
metadata (maximum flat work-group size, static LDS, private segment, VGPRs),
maps the logged addresses to kernel names through the emulated library's
symbol table, and reports every launch that a GPU would not run as written:
more work-items per group than the kernel was compiled for, or static plus
dynamic LDS above the per-group limit.
"""
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LDS_LIMIT = 64 * 1024   # bytes a work-group may allocate without raising the limit


def demangle(names):
    r = subprocess.run(["c++filt"], input="\n".join(names), capture_output=True, text=True, check=True)
    return r.stdout.splitlines()


def norm(s):
    s = s.replace("(anonymous namespace)", "anon").replace(" ", "")
    s = s.replace("longlong", "longlong")
    return s


def device_metadata(csrc, sources, flags=(), out_dir=None):
    """name (demangled, normalised) -> dict of code-object fields, per source."""
    out_dir = out_dir or os.path.join(HERE, "_build", "meta")
    os.makedirs(out_dir, exist_ok=True)
    meta = {}
    for src in sources:
        asm = os.path.join(out_dir, os.path.splitext(src)[0] + ".s")
        cmd = [HIPCC, "-O3", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only", "-S",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *flags,
               os.path.join(csrc, src), "-o", asm]
        subprocess.run(cmd, capture_output=True, text=True, check=True)
        txt = open(asm).read()
        blk = txt[txt.index("amdhsa.kernels"):]
        ents = re.split(r"\n  - ", blk)[1:]
        names, fields = [], []
        for e in ents:
            m = re.search(r"\.name:\s+(\S+)", e)
            if not m:
                continue

            def g(key):
                mm = re.search(r"\." + key + r":\s+(\S+)", e)
                return mm.group(1) if mm else None
            names.append(m.group(1))
            fields.append(dict(mfwg=int(g("max_flat_workgroup_size")), lds=int(g("group_segment_fixed_size")),
                               priv=int(g("private_segment_fixed_size")), vgpr=int(g("vgpr_count")),
                               dynstack=g("uses_dynamic_stack") == "true"))
        for n, d in zip(demangle(names), fields):
            meta[norm(n)] = d
    return meta


def host_symbols(so):
    r = subprocess.run(["nm", "--defined-only", so], capture_output=True, text=True, check=True)
    addr, names = [], []
    for line in r.stdout.splitlines():
        p = line.split()
        if len(p) == 3 and p[1] in "tTwW":
            addr.append(int(p[0], 16))
            names.append(p[2])
    return dict(zip(addr, demangle(names)))


def check(so, log, csrc, sources, flags=()):
    meta = device_metadata(csrc, sources, flags)
    syms = host_symbols(so)
    seen, problems = {}, []
    for line in open(log):
        off, gx, gy, gz, bx, by, bz, shm = [int(v, 16) if i == 0 else int(v) for i, v in enumerate(line.split())]
        name = syms.get(off)
        if name is None:
            problems.append("launch of an unknown kernel at +0x%x" % off)
            continue
        key = norm(name)
        md = meta.get(key)
        if md is None:
            problems.append("no gfx950 metadata for %s" % name)
            continue
        nt = bx * by * bz
        rec = seen.setdefault(key, dict(name=name, md=md, shapes=set()))
        rec["shapes"].add((gx, gy, gz, bx, by, bz, shm))
        if nt > md["mfwg"]:
            problems.append("%s: %d work-items per group, compiled for at most %d" % (name, nt, md["mfwg"]))
        if md["lds"] + shm > LDS_LIMIT:
            problems.append("%s: %d B static + %d B dynamic LDS > %d" % (name, md["lds"], shm, LDS_LIMIT))
        if md["dynstack"]:
            problems.append("%s uses a dynamic stack" % name)
    return seen, problems


def main(argv):
    so, log, csrc = argv[1], argv[2], argv[3]
    sources = argv[4].split(",") if len(argv) > 4 else ["capi.hip", "film.hip", "bulk.hip"]
    seen, problems = check(so, log, csrc, sources)
    for rec in seen.values():
        md = rec["md"]
        print("%-100s mfwg %4d lds %6d priv %4d vgpr %3d  launches %s" %
              (rec["name"][:100], md["mfwg"], md["lds"], md["priv"], md["vgpr"], sorted(rec["shapes"])[:3]))
    for p in problems:
        print("PROBLEM:", p)
    print("LIMITS_DONE problems=%d" % len(problems))
    return 1 if problems else 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))

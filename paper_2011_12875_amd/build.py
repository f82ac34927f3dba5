"""Build the HIP library libsnapmi.so in-tree with hipcc for gfx950.

Each translation unit is compiled to an object in parallel, then linked.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsnapmi.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# (source, extra defines, object name)
UNITS = [
    ("snap_abi.cpp", [], "snap_abi.o"),
    ("snap_tables.cpp", [], "snap_tables.o"),
    ("snap_u.hip", [], "snap_u.o"),
    ("snap_y.hip", [], "snap_y.o"),
    ("snap_dedr.hip", ["-DSNAP_DEDR_LOW"], "snap_dedr_low.o"),
    ("snap_dedr.hip", [], "snap_dedr_high.o"),
    ("snap_dedr_gen.hip", [], "snap_dedr_gen.o"),
    ("snap_misc.hip", [], "snap_misc.o"),
    ("snap_mlp.hip", [], "snap_mlp.o"),
    ("snap_static.hip", [], "snap_static.o"),
]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def _compile(args):
    src, defs, obj, outdir = args
    cmd = [HIPCC] + FLAGS + defs + ["-I", os.path.join(HERE, "..", "include"), "-c",
                                    os.path.join(CSRC, src), "-o", os.path.join(outdir, obj)]
    p = subprocess.run(cmd, capture_output=True, text=True)
    msg = "\n".join(l for l in (p.stdout + p.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in l and l.strip())
    return src, p.returncode, msg, cmd


def build(verbose: bool = False, jobs: int | None = None) -> str:
    """Compile every unit and link libsnapmi.so (always recompiles)."""
    jobs = jobs or min(len(UNITS), max(1, os.cpu_count() or 1))
    with tempfile.TemporaryDirectory(prefix="snapmi_build_") as outdir:
        with cf.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_compile, [(s, d, o, outdir) for s, d, o in UNITS]))
        failed = False
        for src, rc, msg, cmd in results:
            if verbose or rc:
                if msg:
                    print("[%s]\n%s" % (src, msg), flush=True)
            if rc:
                print("compile failed: " + " ".join(cmd), file=sys.stderr)
                failed = True
        if failed:
            raise RuntimeError("libsnapmi build failed")
        tmp = LIB + ".tmp%d" % os.getpid()
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + \
            [os.path.join(outdir, o) for _, _, o in UNITS] + ["-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.check_call(link)
        os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)

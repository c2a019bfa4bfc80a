"""Build libshvis.so for gfx950 in-tree (hipcc, no JIT cache).

Steps: generate the constant tables and unrolled SH-product code
(csrc/gen_tables.py), compile each HIP translation unit to an object in
parallel, link a shared library next to this file; also build the VALU
issue-rate probe (csrc/valu_rate_probe.hip) next to it.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libshvis.so")
# (source, extra flags, object name): the band-count-dependent kernels are
# compiled once per band count.
SOURCES = [("shv_nb.hip", [f"-DSHV_NB={n}", f"-DSHV_PART={part}"], f"shv_nb{n}_p{part}.o")
           for n in range(8, 0, -1) for part in (3, 7, 8, 2, 5, 4, 6, 1, 0)] + [
    ("shv_api.hip", [], "shv_api.o"), ("shv_common.hip", [], "shv_common.o"), ("shv_deform.hip", [], "shv_deform.o"),
    ("shv_raster.hip", [], "shv_raster.o")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled on purpose (see the design notes).
HIPFLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-command-line-argument",
]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed: " + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def _newest_input():
    names = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".h"))]
    names += [os.path.join(CSRC, "generated", f) for f in os.listdir(os.path.join(CSRC, "generated"))]
    names += [os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))]
    names.append(os.path.abspath(__file__))
    return max(os.path.getmtime(n) for n in names)


def build(verbose: bool = False, jobs: int = 8, incremental: bool = False) -> str:
    """Compile everything (``incremental`` skips objects newer than every
    source and header; meant for development only)."""
    os.makedirs(BUILD, exist_ok=True)
    gen_dir = os.path.join(CSRC, "generated")
    gen_stamp = os.path.join(gen_dir, "shv_gaunt.h")
    if not (incremental and os.path.exists(gen_stamp)
            and os.path.getmtime(gen_stamp) >= os.path.getmtime(os.path.join(CSRC, "gen_tables.py"))):
        _run([sys.executable, os.path.join(CSRC, "gen_tables.py"), gen_dir])
    newest = _newest_input()
    objs = []

    def compile_one(entry):
        src, extra, name = entry
        obj = os.path.join(BUILD, name)
        if incremental and os.path.exists(obj) and os.path.getmtime(obj) >= newest:
            return obj
        cmd = [HIPCC, *HIPFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        out = _run(cmd)
        if verbose and out.strip():
            print(out)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    # The VALU issue-rate probe (a measurement tool, not part of the library).
    _run([HIPCC, *HIPFLAGS, os.path.join(CSRC, "valu_rate_probe.hip"), "-o", os.path.join(HERE, "valu_rate_probe")])
    # The FP32 MFMA probe: rounding, lane layout and issue rate (also a measurement tool).
    _run([HIPCC, *HIPFLAGS, os.path.join(CSRC, "mfma_probe.hip"), "-o", os.path.join(HERE, "mfma_probe")])
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))

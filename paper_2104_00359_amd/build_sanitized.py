"""Host-sanitized build of libshvis.so for CPU testing (not the product build).

The translation units that carry the C ABI's host code (argument checks,
workspace carving, work-table packing, graph set-up, the deformation-graph and
incidence builders) are compiled again with AddressSanitizer and
UndefinedBehaviorSanitizer on their host side only (each sanitizer flag right
after -Xarch_host: the GPU code is built as usual), and linked with the
product build's other objects into a library of its own.  Load it with the
sanitizer runtime preloaded (``runtime()``) and SHV_LIBRARY pointing at it.
Needs the objects of a product build (build.py) in _build/.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build  # noqa: E402  (the product build's sources and flags)

OUT = os.path.join(build.BUILD, "sanitize")
LIB = os.path.join(OUT, "libshvis.so")
HOST_UNITS = ("shv_api.hip", "shv_common.hip", "shv_deform.hip", "shv_raster.hip")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined", "-g"]


def runtime() -> str:
    """Path of the AddressSanitizer runtime (it carries UBSan's handlers too)."""
    return subprocess.run([build.HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], stdout=subprocess.PIPE,
                          text=True, check=True).stdout.strip()


def build_sanitized(jobs: int = 8) -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for src, extra, name in build.SOURCES:
        obj = os.path.join(build.BUILD, name)
        if src in HOST_UNITS:
            continue
        if not os.path.exists(obj):
            raise FileNotFoundError(f"{obj} is missing: run the product build first")
        objs.append(obj)

    def compile_one(src):
        obj = os.path.join(OUT, src.replace(".hip", ".o"))
        build._run([build.HIPCC, *build.HIPFLAGS, *SAN, "-c", os.path.join(build.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs += list(ex.map(compile_one, HOST_UNITS))
    build._run([build.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libasan", *SAN[:4], "-o", LIB,
                *objs])
    return LIB


if __name__ == "__main__":
    print(build_sanitized())

"""Host-sanitizer build of the library's host code, for the tests.

The planner, the field code and the C-ABI layer (csrc/plan.cpp, field.cpp,
api.cpp) are compiled with g++ and AddressSanitizer + UndefinedBehaviorSanitizer,
then linked with the device objects of the ordinary build (csrc/_build/*.o from
build.py, whose kernels are not instrumented) into libffa_hostsan.so.  Loading it
needs the ASan runtime first in the process (LD_PRELOAD of gcc's libasan) and
FFA_LIBRARY pointing at it.

    python -m paper_2101_01025_amd.build_host_sanitized OUTDIR
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(CSRC, "_build")
HOST_SOURCES = ["field.cpp", "plan.cpp", "api.cpp"]
DEVICE_OBJECTS = ["gemm_i8_part_a.o", "gemm_i8_part_b.o", "gemm_i8_part_c.o", "gemm_i8_part_d.o",
                  "gemm_i8_part_e.o", "gemm_i8.o", "gemm_f64.o", "elementwise.o", "noalloc.o"]
ROCM = "/opt/rocm"
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"]


def device_objects():
    objs = [os.path.join(OBJDIR, o) for o in DEVICE_OBJECTS]
    missing = [o for o in objs if not os.path.exists(o)]
    if missing:
        raise FileNotFoundError(f"device objects of the ordinary build are missing: {missing}")
    return objs


def build(outdir: str) -> str:
    os.makedirs(outdir, exist_ok=True)
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(outdir, os.path.splitext(src)[0] + ".o")
        subprocess.check_call(["g++", "-O1", "-g", "-fPIC", "-std=c++17", *SAN,
                               "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include", "-c",
                               os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    lib = os.path.join(outdir, "libffa_hostsan.so")
    subprocess.check_call(["g++", "-shared", *SAN, "-o", lib, *objs, *device_objects(),
                           f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{ROCM}/lib"])
    return lib


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else os.path.join(OBJDIR, "hostsan")))

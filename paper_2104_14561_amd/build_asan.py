"""AddressSanitizer build of the library's host code (CPU checks only).

fk_host.cpp (plan construction, validation, layout, the work lists) is
compiled with AddressSanitizer on the host side only and linked with the
device objects of the ordinary build into _build/asan/libfkexit_asan.so.  The
sanitizer runtime is not linked into the library: a process loads it with
LD_PRELOAD (runtime_path()).  Device code is never instrumented."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

from . import build as B

ASAN_DIR = os.path.join(B.HERE, "_build", "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libfkexit_asan.so")


def runtime_path() -> str:
    """The clang AddressSanitizer runtime that matches hipcc's compiler."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(B.hipcc())))
    hits = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang AddressSanitizer runtime not found")
    return hits[-1]


def build_asan() -> str:
    """Compile fk_host.cpp with host-side AddressSanitizer and link it with the
    device objects of the ordinary build (built first if missing)."""
    names = [name for _, name, _ in B.units() if name != "fk_host"]
    objs = [os.path.join(B.HERE, "_build", n + ".o") for n in names]
    if not all(os.path.exists(o) for o in objs):
        B.build()
    os.makedirs(ASAN_DIR, exist_ok=True)
    host_obj = os.path.join(ASAN_DIR, "fk_host.o")
    cmd = ([B.hipcc()] + B.compile_flags() +
           ["-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer", "-g",
            "-c", os.path.join(B.CSRC, "fk_host.cpp"), "-o", host_obj])
    subprocess.check_call(cmd)
    tmp = ASAN_LIB + ".tmp"
    subprocess.check_call([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC",
                           "-o", tmp, host_obj] + objs)
    os.replace(tmp, ASAN_LIB)
    return ASAN_LIB


if __name__ == "__main__":
    print(build_asan())
    sys.stdout.flush()

"""Build libfkexit.so (HIP, gfx950) in-tree with hipcc.

The kernels are split over several translation units: fk_launch.hip (slope
pass, lane-group kernels, ELL form, exports) and one instance of
fk_node_inst.hip per (precision, dimension, forward|adjoint), each holding the
thread-per-node and separable-box specialisations over Q*.  They compile in
parallel."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfkexit.so")
ARCH = os.environ.get("FKEXIT_ARCH", "gfx950")


def units():
    """(source, object name, extra defines) of every translation unit."""
    out = [("fk_host.cpp", "fk_host", []), ("fk_launch.hip", "fk_launch", [])]
    for adj in (0, 1):
        for f32 in (1, 0):
            for d in (2, 3, 1):
                name = f"{'adjoint' if adj else 'step'}_node_{'f32' if f32 else 'f64'}_d{d}"
                out.append(("fk_node_inst.hip", name,
                            [f"-DFK_INST_F32={f32}", f"-DFK_INST_D={d}", f"-DFK_INST_ADJ={adj}",
                             f"-DFK_INST_NAME={name}"]))
    return out


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        # packed FP32 instructions are kept out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        # hardware floating-point atomics (adjoint scatter)
        "-munsafe-fp-atomics",
        "-I", INCLUDE, "-I", CSRC,
    ]


def _jobs() -> int:
    env = os.environ.get("MAX_JOBS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return max(1, min(16, os.cpu_count() or 1))


def build(verbose: bool = False) -> str:
    """Compile every translation unit to an object (in parallel), then link."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    jobs = []
    for src, name, defs in units():
        obj = os.path.join(bdir, name + ".o")
        cmd = [hipcc()] + compile_flags() + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
        jobs.append((cmd, obj))

    def run(job):
        cmd, obj = job
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return cmd, obj, r.returncode, r.stdout

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        results = list(ex.map(run, jobs))
    failed = [(cmd, out) for cmd, _, rc, out in results if rc != 0]
    for cmd, out in failed:
        print(" ".join(cmd), file=sys.stderr)
        print(out, file=sys.stderr)
    if failed:
        raise RuntimeError(f"{len(failed)} translation unit(s) failed to compile")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + [o for _, o, _, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)

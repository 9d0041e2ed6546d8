"""The library's host code under AddressSanitizer (CPU only, no kernel runs).

fk_host.cpp is compiled with host-side AddressSanitizer and linked with the
ordinary device objects (paper_2104_14561_amd/build_asan.py); a child process
loads the sanitizer runtime with LD_PRELOAD and the instrumented library
through FKEXIT_LIB, then
  * runs the host-only ABI suite (tests/test_abi_cpu.py), and
  * creates, inspects and destroys plans of every problem family and option
    the host code branches on (batched uneven 2D grids, 3D periodic axes, the
    assembled form, checkpointed adjoint lists, FP64 child plans, the R2
    interpolant, boundary faces, the runaway-electron model, 1D).
A heap overflow, use after free or double free in that code aborts the child
with the sanitizer's report, which the assertion prints."""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "paper_2104_14561_amd", "csrc", f)
           for f in ("fk_host.cpp", "fk_internal.h")] + [os.path.join(ROOT, "include", "fkexit.h")]

PLANS = r"""
import ctypes, sys
import numpy as np
import workloads as W
from paper_2104_14561_amd import fkexit
lib = fkexit.load()
assert fkexit.LIB_PATH.endswith("libfkexit_asan.so"), fkexit.LIB_PATH
maps = open("/proc/self/maps").read()
assert "libfkexit_asan.so" in maps and "libclang_rt.asan" in maps

def plan(probs, force=None, **opt):
    arr, keep = fkexit._marshal(probs, force)
    o = fkexit._Options()
    o.precision = fkexit.PREC[opt.get("precision", "f32")]
    o.form = fkexit.FORM[opt.get("form", "fused")]
    o.ckpt_every = opt.get("ckpt_every", 0)
    o.hermite = fkexit.HERMITE[opt.get("hermite", "r1")]
    h = ctypes.c_void_p()
    st = lib.fk_plan_create(arr, len(probs), ctypes.byref(o), ctypes.byref(h))
    assert st == 0, (st, lib.fk_last_error().decode())
    info = fkexit._Info()
    assert lib.fk_plan_get_info(h, ctypes.byref(info)) == 0
    off = (ctypes.c_int64 * (len(probs) + 1))()
    cnt = (ctypes.c_int64 * len(probs))()
    assert lib.fk_plan_layout(h, off, cnt) == 0
    assert off[len(probs)] == info.n_nodes and sum(cnt) == info.n_active
    lib.fk_plan_destroy(h)
    return info

batch = W.cell2d_batch(n_inst=6, n_steps=4)
plan(batch)
plan(batch, ckpt_every=2)
plan(batch, ckpt_every=1, force=[i % 2 for i in range(len(batch))])
plan(batch, precision="f64", form="ell")
plan([batch[0].replace(hermite="r2")], precision="f64", hermite="r2")
abc = W.abc3d_batch(n_inst=2, n=17, n_steps=2)
plan(abc, ckpt_every=1)
plan(abc, precision="f64", ckpt_every=2, force=[1, 0])
plan([W.paper2d(n1=33, n2=17).replace(n_steps=3)], ckpt_every=1)
plan([W.runaway3d(n_p=9, n_xi=9, T=1.0)], precision="f64")
plan([W.bm1d(n=41, n_steps=3)], precision="f64", ckpt_every=1)
plan([W.bm1d(n=41, n_steps=3)], form="ell")
print("plans ok", flush=True)
"""


@pytest.fixture(scope="module")
def asan_env():
    from paper_2104_14561_amd import build as B
    from paper_2104_14561_amd import build_asan as BA
    try:
        B.hipcc()
        rt = BA.runtime_path()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = BA.ASAN_LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(s) for s in SOURCES):
        BA.build_asan()
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, FKEXIT_LIB=lib,
               # Python and torch allocate for the life of the process
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    return env


def _run(cmd, env):
    r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=600)
    assert r.returncode == 0 and "AddressSanitizer" not in r.stdout, r.stdout[-6000:]
    return r.stdout


def test_library_is_instrumented(asan_env):
    # the instrumented host code calls the sanitizer's report hooks
    with open(asan_env["FKEXIT_LIB"], "rb") as fh:
        assert b"__asan_report_load8" in fh.read()


def test_abi_suite_under_asan(asan_env):
    out = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                os.path.join("tests", "test_abi_cpu.py")], asan_env)
    assert " passed" in out


def test_plan_lifecycle_of_every_family_under_asan(asan_env):
    assert "plans ok" in _run([sys.executable, "-c", PLANS], asan_env)

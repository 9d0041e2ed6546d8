"""Host-only checks of the C ABI: the library loads, exports every symbol that
include/fkexit.h declares, validates problems and computes its own
Gauss-Hermite rule.  Nothing here launches a kernel."""
from __future__ import annotations

import ctypes
import math
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2104_14561_amd import fkexit

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "fkexit.h")).read()
    return sorted(set(re.findall(r"\b(fk_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fkexit.LIB_PATH):
        pytest.skip("libfkexit.so not built")
    return fkexit.load()


def test_exports_every_declared_symbol(lib):
    syms = _declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(fkexit.EXPORTED)
    txt = open(os.path.join(ROOT, "include", "fkexit.h")).read()
    version = int(re.search(r"#define FK_ABI_VERSION (\d+)", txt).group(1))
    assert lib.fk_version() == version


@pytest.mark.parametrize("q", [1, 2, 3, 6, 8, 16, 32, 64])
def test_library_gh_rule(q, lib):
    a, w = fkexit.gh_rule(q)
    ha, hw = np.polynomial.hermite.hermgauss(q)
    np.testing.assert_allclose(a, ha, atol=5e-13 * max(1.0, np.abs(ha).max()))
    np.testing.assert_allclose(w, hw / math.sqrt(math.pi), rtol=1e-10, atol=1e-15)
    assert abs(w.sum() - 1.0) < 1e-13
    assert np.all(a == -a[::-1])


def test_library_gh_matches_oracle_nodes(lib):
    """Two independent rules (Sturm bisection + Newton vs Golub-Welsch eigen)
    agree to a few ulps; exact ties (the zero node of odd rules) coincide."""
    import oracle
    for q in (3, 6, 8, 16):
        a, _ = fkexit.gh_rule(q)
        b, _ = oracle.gh_rule(q)
        assert np.abs(a - b).max() <= 4 * np.spacing(np.abs(b).max())
        if q % 2:
            assert a[q // 2] == 0.0 and b[q // 2] == 0.0


def _create(problems, **opt):
    lib = fkexit.load()
    arr, keep = fkexit._marshal(problems)
    o = fkexit._Options()
    o.precision = fkexit.PREC[opt.get("precision", "f64")]
    o.form = fkexit.FORM[opt.get("form", "fused")]
    o.ckpt_every = opt.get("ckpt_every", 0)
    h = ctypes.c_void_p()
    st = lib.fk_plan_create(arr, len(problems), ctypes.byref(o), ctypes.byref(h))
    return st, h, lib.fk_last_error().decode()


def test_plan_info_and_layout(lib):
    probs = W.cell2d_batch(n_inst=4, n_steps=3)
    st, h, msg = _create(probs, precision="f32")
    assert st == 0, msg
    info = fkexit._Info()
    assert lib.fk_plan_get_info(h, ctypes.byref(info)) == 0
    assert info.n_inst == 4 and info.d == 2 and info.n_quad == 64 and info.n_theta == 4
    assert info.n_nodes == sum(p.n_nodes for p in probs)
    off = (ctypes.c_int64 * 5)()
    cnt = (ctypes.c_int64 * 4)()
    assert lib.fk_plan_layout(h, off, cnt) == 0
    assert list(off)[-1] == info.n_nodes and sum(cnt) == info.n_active
    import oracle
    for i, p in enumerate(probs):
        assert cnt[i] == oracle.active_nodes(p).shape[0]
    assert info.workspace_bytes > 0
    lib.fk_plan_destroy(h)


def test_active_set_matches_oracle_on_periodic_3d(lib):
    import oracle
    p = W.abc3d(n=17, n_steps=2)
    st, h, msg = _create([p], precision="f32")
    assert st == 0, msg
    cnt = (ctypes.c_int64 * 1)()
    lib.fk_plan_layout(h, None, cnt)
    assert cnt[0] == oracle.active_nodes(p).shape[0] == 16 * 16 * 15
    lib.fk_plan_destroy(h)


@pytest.mark.parametrize("case,status", [
    ("d0", -1), ("n3", -1), ("nonincreasing", -1), ("nan_coef", -5), ("neg_D", -1),
    ("dt0", -1), ("q0", -1), ("ball_outside", -1), ("mismatch", -1), ("ell_periodic", -2),
    ("adj_D0", -1), ("bad_prec", -1),
])
def test_validation_errors(lib, case, status):
    base = W.cell2d(nx=33, ny=17, n_steps=2)
    probs, opt = [base], {}
    if case == "d0":
        probs = [base.replace(axes=[])]
    elif case == "n3":
        probs = [base.replace(axes=[W.uniform_axis(0, 2, 3), base.axes[1]])]
    elif case == "nonincreasing":
        x = base.axes[0].nodes.copy()
        x[5] = x[4]
        probs = [base.replace(axes=[W.Axis(x), base.axes[1]])]
    elif case == "nan_coef":
        probs = [base.replace(coef=(float("nan"), 0.1, 1.0))]
    elif case == "neg_D":
        probs = [base.replace(D=-1.0)]
    elif case == "dt0":
        probs = [base.replace(dt=0.0)]
    elif case == "q0":
        probs = [base.replace(gh_q=0)]
    elif case == "ball_outside":
        probs = [base.replace(radius=0.6)]
    elif case == "mismatch":
        probs = [base, base.replace(n_steps=3)]
    elif case == "ell_periodic":
        probs, opt = [W.abc3d(n=9, n_steps=2)], {"form": "ell"}
    elif case == "adj_D0":
        probs, opt = [base.replace(D=0.0)], {"ckpt_every": 4}
    elif case == "bad_prec":
        opt = {"precision": "f64"}
    if case == "bad_prec":
        lib_ = fkexit.load()
        arr, keep = fkexit._marshal(probs)
        o = fkexit._Options()
        o.precision = 7
        h = ctypes.c_void_p()
        st = lib_.fk_plan_create(arr, 1, ctypes.byref(o), ctypes.byref(h))
        msg = lib_.fk_last_error().decode()
    else:
        st, h, msg = _create(probs, **opt)
    assert st == status, (case, st, msg)
    assert msg


def test_calls_without_workspace_fail_cleanly(lib):
    st, h, msg = _create([W.bm1d()])
    assert st == 0
    snaps = (ctypes.c_int * 1)(0)
    assert lib.fk_forward(h, snaps, 1, None, None) == -6
    assert "workspace" in lib.fk_last_error().decode()
    lib.fk_plan_destroy(h)


def test_workspace_too_small_rejected(lib):
    st, h, msg = _create([W.bm1d()])
    assert st == 0
    info = fkexit._Info()
    lib.fk_plan_get_info(h, ctypes.byref(info))
    # a fake aligned pointer: the size check happens before any device access
    assert lib.fk_plan_set_workspace(h, ctypes.c_void_p(1 << 20), info.workspace_bytes - 1,
                                     None) == -3
    assert lib.fk_plan_set_workspace(h, ctypes.c_void_p((1 << 20) + 8), info.workspace_bytes,
                                     None) == -1
    lib.fk_plan_destroy(h)


def test_tune_rejects_bad_arguments(lib):
    """fk_tune validates its arguments on the host before touching a device."""
    arr, keep = fkexit._marshal([W.bm1d()])
    res = fkexit._TuneResult()
    opt = fkexit._Options()
    # no problems
    assert lib.fk_tune(None, 0, ctypes.byref(opt), 4, None, 0, None, ctypes.byref(res)) == -1
    # no result
    assert lib.fk_tune(arr, 1, ctypes.byref(opt), 4, ctypes.c_void_p(256), 1 << 20, None, None) == -1
    # trial_steps < 1
    assert lib.fk_tune(arr, 1, ctypes.byref(opt), 0, ctypes.c_void_p(256), 1 << 20, None,
                       ctypes.byref(res)) == -1
    # no workspace
    assert lib.fk_tune(arr, 1, ctypes.byref(opt), 4, None, 0, None, ctypes.byref(res)) == -1
    assert "workspace" in lib.fk_last_error().decode()
    del keep


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why,
    before touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout

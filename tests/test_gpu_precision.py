"""Instances forced to FP64 inside an FP32 plan (fk_problem.force_f64) and the
precision probe (fk_probe_precision), through the C ABI.

A forced instance is computed by the same FP64 kernels as an FP64 plan, so
its FP32 outputs are that plan's results rounded to FP32 (bitwise); the other
instances are computed by the same FP32 kernels as a plain FP32 plan (bitwise,
same step layout).  Covered: snapshots, a resumed pass, one step from a
caller state, the adjoint (gradient rows and dJ/du^N), landing cells, and the
probe's per-instance differences and flags.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import FkError, Plan, precision_probe  # noqa: E402


def _batch():
    return [W.cell2d(nx=65, ny=33, n_steps=40, D=2e-3, A=0.9),
            W.cell2d(nx=97, ny=49, n_steps=40, D=1e-3, A=1.2, eps=0.2),
            W.cell2d(nx=129, ny=65, n_steps=40, D=4e-3, A=0.7, omega=9.0)]


FORCE = [False, True, False]


def _np(t):
    return t.double().cpu().numpy()


def test_forced_instances_forward_and_step():
    probs = _batch()
    snaps = [40, 23, 0]
    mixed = Plan(probs, precision="f32", step_kernel="node", force_f64=FORCE)
    p32 = Plan(probs, precision="f32", step_kernel="node")
    p64 = Plan(probs, precision="f64", step_kernel="node")
    assert mixed.info.n_active == p32.info.n_active
    assert mixed.active_count == p32.active_count
    got = mixed.forward(snaps)
    r32 = p32.forward(snaps)
    r64 = p64.forward(snaps)
    torch.cuda.synchronize()
    assert mixed.check_flags() == 0
    g, a, b = mixed.split(got), p32.split(r32), p64.split(r64)
    for i, f in enumerate(FORCE):
        want = b[i].float() if f else a[i]
        assert torch.equal(g[i], want), i
    # resumed from a caller state, and one step from it
    u_mid = got[1].clone()
    res = mixed.split(mixed.forward_from(u_mid, 23, [0]))
    res32 = p32.split(p32.forward_from(u_mid, 23, [0]))
    res64 = p64.split(p64.forward_from(u_mid.double(), 23, [0]))
    for i, f in enumerate(FORCE):
        want = res64[i].float() if f else res32[i]
        assert torch.equal(res[i], want), i
    one = mixed.step(22, u_mid)
    one32 = p32.step(22, u_mid)
    one64 = p64.step(22, u_mid.double())
    torch.cuda.synchronize()
    s1, s2, s3 = mixed.split(one), p32.split(one32), p64.split(one64)
    for i, f in enumerate(FORCE):
        want = s3[i].float() if f else s2[i]
        assert torch.equal(s1[i], want), i
    # landing cells of the forced instance come from its FP64 plan
    c_m, e_m = mixed.export_cells(1, 5)
    c_o, e_o = oracle.step_cells(probs[1], 5, oracle.chi(probs[1]))
    torch.cuda.synchronize()
    assert np.array_equal(c_m.cpu().numpy(), c_o) and np.array_equal(e_m.cpu().numpy(), e_o)
    for p in (mixed, p32, p64):
        p.close()


def test_forced_instances_adjoint():
    probs = _batch()
    lam0 = torch.cat([torch.from_numpy(W.region_mean_weights(p).reshape(-1)) for p in probs])
    mixed = Plan(probs, precision="f32", step_kernel="node", force_f64=FORCE, ckpt_every=8)
    p32 = Plan(probs, precision="f32", step_kernel="node", ckpt_every=8)
    p64 = Plan(probs, precision="f64", step_kernel="node", ckpt_every=8)
    gm, lm = mixed.adjoint(lam0)
    g32, l32 = p32.adjoint(lam0)
    # the FP32 plan takes its cotangent in FP32: the FP64 reference gets the
    # same rounded values
    g64, l64 = p64.adjoint(lam0.float().double())
    torch.cuda.synchronize()
    gm, g32, g64 = _np(gm), _np(g32), _np(g64)
    for i, f in enumerate(FORCE):
        want = g64[i] if f else g32[i]
        rel = np.abs(gm[i] - want).max() / np.abs(want).max()
        print(f"instance {i} forced={f}: grad rel diff {rel:.2e}")
        # atomics order the scatter differently run to run
        assert rel <= (1e-12 if f else 1e-5)
    sm, s32, s64 = mixed.split(lm), p32.split(l32), p64.split(l64)
    for i, f in enumerate(FORCE):
        want = s64[i].float() if f else s32[i]
        scale = float(want.abs().max())
        err = float((sm[i] - want).abs().max())
        assert err <= (1e-6 if f else 1e-4) * scale, (i, err, scale)
    for p in (mixed, p32, p64):
        p.close()


def test_forced_instances_refused_where_unsupported():
    probs = _batch()
    with pytest.raises(FkError, match="FK_ERR_UNSUPPORTED"):
        Plan(probs, precision="f32", form="ell", force_f64=FORCE)
    mixed = Plan(probs, precision="f32", force_f64=FORCE, ckpt_every=4)
    with pytest.raises(FkError, match="FK_ERR_UNSUPPORTED"):
        mixed.forward_static([0])
    with pytest.raises(FkError, match="FK_ERR_UNSUPPORTED"):
        mixed.apply_step(0, torch.zeros(3 * mixed.n_nodes))
    mixed.close()
    # in an FP64 plan the flag changes nothing
    pa = Plan(probs, precision="f64", step_kernel="node", force_f64=FORCE)
    pb = Plan(probs, precision="f64", step_kernel="node")
    a, b = pa.forward([0]), pb.forward([0])
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    pa.close()
    pb.close()


def test_precision_probe_matches_separate_passes():
    probs = _batch()
    tol = 1e-7
    flags, diffs, _ = precision_probe(probs, tol=tol, step_kernel="node")
    p64 = Plan(probs, precision="f64", step_kernel="node")
    p32 = Plan(probs, precision="f32", step_kernel="node")
    r64, r32 = p64.forward([0])[0], p32.forward([0])[0]
    torch.cuda.synchronize()
    d = [float((a - b.double()).abs().max()) for a, b in zip(p64.split(r64), p32.split(r32))]
    p64.close()
    p32.close()
    print("probe diffs", diffs, "separate", d, "flags", flags)
    assert np.allclose(diffs, d, rtol=0, atol=0)
    assert flags == [x > tol / 2 for x in d]


def test_precision_probe_gradients():
    """With a cotangent the probe also compares the FP64 and FP32 adjoints:
    its relative gradient differences equal those of separate plans (up to
    the atomics' summation order) and flag instances beyond grad_tol / 2."""
    probs = _batch()
    lam0 = torch.cat([torch.from_numpy(W.region_mean_weights(p).reshape(-1)) for p in probs])
    flags, diffs, gd = precision_probe(probs, tol=1.0, lam0=lam0, grad_tol=2e-6,
                                       step_kernel="node")
    p64 = Plan(probs, precision="f64", step_kernel="node", ckpt_every=32)
    p32 = Plan(probs, precision="f32", step_kernel="node", ckpt_every=32)
    g64 = p64.adjoint(lam0)[0].cpu().numpy()
    g32 = p32.adjoint(lam0.float())[0].cpu().numpy()
    p64.close()
    p32.close()
    ref = [float(np.abs(a - b).max() / np.abs(a).max()) for a, b in zip(g64, g32)]
    print("probe grad diffs", gd, "separate", ref, "flags", flags)
    # the FP32 adjoint's scatter order varies run to run (atomics): about
    # 1e-8 of the gradient, i.e. about 1 % of a 1e-6 difference
    for a, b in zip(gd, ref):
        assert abs(a - b) <= 0.05 * b + 1e-12
    assert flags == [x > 1e-6 for x in gd]

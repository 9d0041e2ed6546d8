"""The R2 interpolant (full tensor cubic Hermite with the PCHIP-composed
twist fields, Section 3.1.2) on the GPU against the oracle's R2: fields of
the time-dependent cellular flow (disc exit) and of the paper's periodic
roll flow, FP64 within 1e-12 and FP32 within 1e-5, every 2D step layout;
in 3D the ABC flow (periodic x, y) with its four twist fields, both
thread-per-node layouts; R2 and R1 differ by far more than the bars (the
twists enter); Algorithm 1 with R2; the combinations outside what is built
are refused."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import FkError, Plan  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5}


def _cases():
    return {"cell2d": W.cell2d(nx=97, ny=49, n_steps=40, D=2e-3).replace(hermite="r2"),
            "paper2d": W.paper2d(n1=65, n2=17).replace(n_steps=40, hermite="r2")}


@pytest.mark.parametrize("kernel", ["node", "group", "split", "box"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["cell2d", "paper2d"])
def test_r2_fields_match_oracle(name, prec, kernel):
    prob = _cases()[name]
    snaps = [prob.n_steps, 17, 0]
    ref = oracle.solve(prob, snaps=snaps)
    plan = Plan(prob, precision=prec, step_kernel=kernel, hermite="r2", use_graph=True)
    got = plan.split(plan.forward(snaps))[0].double().cpu().numpy()
    torch.cuda.synchronize()
    assert plan.check_flags() == 0
    plan.close()
    err = float(np.abs(got - ref).max())
    r1 = oracle.solve(prob.replace(hermite="r1"), snaps=[0])[0]
    gap = float(np.abs(ref[-1] - r1).max())
    print(f"R2 {name} {prec} {kernel}: max|gpu - oracle| {err:.3e} (R2 - R1: {gap:.2e})")
    assert err <= TOL[prec]
    assert gap > 10 * TOL[prec]


def _abc_r2():
    # a coarse grid and a step long enough that landing points sit well
    # inside their cells, where the twist terms matter
    return W.abc3d(n=17, D=1e-2, dt=0.05, n_steps=8).replace(hermite="r2")


@pytest.mark.parametrize("kernel", ["node", "split"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_r2_3d_fields_match_oracle(prec, kernel):
    prob = _abc_r2()
    snaps = [prob.n_steps, 3, 0]
    ref = oracle.solve(prob, snaps=snaps)
    plan = Plan(prob, precision=prec, step_kernel=kernel, hermite="r2", use_graph=True)
    got = plan.split(plan.forward(snaps))[0].double().cpu().numpy()
    torch.cuda.synchronize()
    assert plan.check_flags() == 0
    plan.close()
    err = float(np.abs(got - ref).max())
    r1 = oracle.solve(prob.replace(hermite="r1"), snaps=[0])[0]
    gap = float(np.abs(ref[-1] - r1).max())
    print(f"R2 abc3d {prec} {kernel}: max|gpu - oracle| {err:.3e} (R2 - R1: {gap:.2e})")
    assert err <= TOL[prec]
    assert gap > 10 * TOL[prec]


def test_r2_3d_batched_uneven_and_single_step():
    a = _abc_r2()
    b = W.abc3d(n=13, D=2e-2, dt=0.05, n_steps=8).replace(hermite="r2")
    plan = Plan([a, b], precision="f64", hermite="r2")
    got = plan.split(plan.forward([0]))
    torch.cuda.synchronize()
    for g, p in zip(got, (a, b)):
        assert np.abs(g[0].cpu().numpy() - oracle.solve(p, snaps=[0])[0]).max() <= 1e-12
    plan.close()
    u = W.random_field(a.shape, seed=5)
    plan = Plan(a, precision="f64", hermite="r2")
    got = plan.step(2, torch.from_numpy(u.reshape(-1))).cpu().numpy().reshape(a.shape)
    torch.cuda.synchronize()
    plan.close()
    assert np.abs(got - oracle.step(a, 2, u)).max() <= 1e-12


def test_r2_horizons_match_oracle():
    prob = _cases()["cell2d"]
    hz = [40, 9, 25]
    plan = Plan(prob, precision="f64", hermite="r2")
    got = plan.split(plan.forward_horizons(hz))[0].cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    assert np.abs(got - oracle.solve_horizons(prob, hz)).max() <= 1e-12


def test_r2_single_step_from_random_state():
    prob = _cases()["cell2d"]
    u = W.random_field(prob.shape, seed=12)
    plan = Plan(prob, precision="f64", hermite="r2")
    got = plan.step(5, torch.from_numpy(u.reshape(-1))).cpu().numpy().reshape(prob.shape)
    torch.cuda.synchronize()
    plan.close()
    assert np.abs(got - oracle.step(prob, 5, u)).max() <= 1e-12


def test_r2_refused_outside_what_is_built():
    c = _cases()["cell2d"]
    for kw in ({"form": "ell"}, {"ckpt_every": 4}):
        with pytest.raises(FkError, match="FK_ERR_UNSUPPORTED"):
            Plan(c, hermite="r2", **kw)
    # 3D: the twist records are read by the thread-per-node step only
    for kernel in ("group", "box"):
        with pytest.raises(FkError, match="FK_ERR_UNSUPPORTED"):
            Plan(W.abc3d(n=9, n_steps=2).replace(hermite="r2"), hermite="r2", step_kernel=kernel)

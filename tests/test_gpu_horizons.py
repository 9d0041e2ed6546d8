"""Algorithm 1 (Section 3.2, Eq. (e37)) on the GPU through fk_forward_horizons:
several horizons in one backward sweep, the step operator of each sweep index
shared by the columns still running (assembled form: one assembly per index,
applied to up to 4 columns per launch; fused form: the matrix-free step per
column), against the oracle's own Algorithm 1 (fko_solve_horizons): FP64
within 1e-12, FP32 within 1e-5; batched uneven instances; unsorted and
repeated horizons; a column equals the Scheme-1 pass of that many steps."""
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
    return [W.cell2d(nx=97, ny=49, n_steps=60, D=2e-3),
            W.cell2d(nx=65, ny=33, n_steps=60, D=4e-3, A=1.3, eps=0.25, omega=9.0)]


@pytest.mark.parametrize("columns", [1, 3, 4])
@pytest.mark.parametrize("form", ["fused", "ell"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_horizons_match_oracle_algorithm1(prec, form, columns):
    if form == "fused" and columns != 1:
        pytest.skip("columns applies to the assembled product")
    probs = _cases()
    hz = [5, 17, 17, 33, 60, 41, 1]
    plan = Plan(probs, precision=prec, form=form, columns=columns, use_graph=True)
    out = plan.forward_horizons(hz)
    out2 = plan.forward_horizons(hz)      # graph replay
    torch.cuda.synchronize()
    assert plan.check_flags() == 0
    assert torch.equal(out, out2)
    got = plan.split(out)
    worst = 0.0
    for i, prob in enumerate(probs):
        ref = oracle.solve_horizons(prob, hz)
        err = float(np.abs(got[i].double().cpu().numpy() - ref).max())
        worst = max(worst, err)
    plan.close()
    print(f"horizons {prec} {form} columns={columns}: max|gpu - oracle| {worst:.3e}")
    assert worst <= TOL[prec]


def test_horizon_column_equals_scheme1_pass():
    """Column m is the Scheme-1 pass of m steps from t0 (same kernels, same
    per-node arithmetic: bitwise in the fused form)."""
    prob = _cases()[0]
    plan = Plan(prob, precision="f64", step_kernel="node")
    cols = plan.split(plan.forward_horizons([60, 23]))[0]
    short = Plan(prob.replace(n_steps=23), precision="f64", step_kernel="node")
    u23 = short.split(short.forward([0]))[0][0]
    full = plan.split(plan.forward([0]))[0][0]
    torch.cuda.synchronize()
    assert torch.equal(cols[0], full)
    assert torch.equal(cols[1], u23)
    plan.close()
    short.close()


def test_horizons_argument_errors():
    prob = _cases()[0]
    plan = Plan(prob)
    for bad in ([0], [61], []):
        with pytest.raises(FkError, match="FK_ERR_ARG"):
            plan.forward_horizons(bad)
    plan.close()

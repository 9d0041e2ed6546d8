"""fk_forward_static (the allocation-free forward pass on the library's
static device buffer) against fk_forward on a caller workspace, through the C
ABI: two calls in a row, the second on a smaller plan that has no workspace of
its own, FP64 and FP32, results equal to the workspace pass (the kernels and
their order are the same: bitwise); plans too large for the buffer are
refused."""
from __future__ import annotations

import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import FkError, Plan  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5}


def _forward(prob, prec, snaps):
    plan = Plan(prob, precision=prec)
    out = plan.forward(snaps).double().cpu().numpy()
    plan.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_static_forward_matches_workspace_forward(prec):
    big = W.cell2d(nx=257, ny=129, n_steps=40, D=2e-3)
    small = W.cell2d(nx=65, ny=33, n_steps=25, D=3e-3)
    ref_big = _forward(big, prec, [0, 17])
    ref_small = _forward(small, prec, [0, 9])
    p1 = Plan(big, precision=prec, allocate=False)
    got_big = p1.forward_static([0, 17])
    p2 = Plan(small, precision=prec, allocate=False)
    got_small = p2.forward_static([0, 9])
    torch.cuda.synchronize()
    got_big = got_big.double().cpu().numpy()
    got_small = got_small.double().cpu().numpy()
    e1 = float(np.abs(got_big - ref_big).max())
    e2 = float(np.abs(got_small - ref_small).max())
    print(f"static forward {prec}: 257x129 {e1:.3e}, then 65x33 {e2:.3e}", flush=True)
    assert e1 <= TOL[prec] and e2 <= TOL[prec]
    assert np.array_equal(got_big, ref_big) and np.array_equal(got_small, ref_small)
    p1.close()
    p2.close()


def test_static_forward_refuses_large_plans():
    prob = W.abc3d(n=129, n_steps=2)
    plan = Plan(prob, precision="f64", allocate=False)
    with pytest.raises(FkError, match="FK_ERR_WORKSPACE"):
        plan.forward_static([0])
    plan.close()

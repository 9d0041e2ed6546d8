"""The paper's own 2D example (Section 4.2): Pe v of Eq. (ex3) on
[-pi, pi] x [0, 1], periodic in x_1, exit through x_2 = 0 and 1, through the
library's FK_COEF_ROLLS2D kind, against the oracle: fields (FP64 within 1e-12,
FP32 within 1e-5), landing cells bit-exact, the adjoint gradient with respect
to (Pe, eps, omega, D) within 1e-10 relative of the oracle's adjoint, and the
result the paper states for its figure (low exit probability in the roll
cores, high at the separatrices) on the GPU's own field."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import Plan  # noqa: E402

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.mark.parametrize("kernel", ["node", "group", "split", "box"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_paper2d_fields_match_oracle(prec, kernel):
    prob = W.paper2d()
    snaps = [prob.n_steps, 50, 0]
    ref = oracle.solve(prob, snaps=snaps)
    plan = Plan(prob, precision=prec, step_kernel=kernel, use_graph=True)
    got = plan.split(plan.forward(snaps))[0].double().cpu().numpy()
    torch.cuda.synchronize()
    assert plan.check_flags() == 0
    plan.close()
    err = float(np.abs(got - ref).max())
    print(f"paper2d {prec} {kernel}: max|gpu - oracle| {err:.3e}")
    assert err <= TOL[prec]
    u0 = got[-1]
    x1, x2 = prob.axes[0].nodes, prob.axes[1].nodes
    mid = int(np.argmin(np.abs(x2 - 0.5)))
    at = lambda v: u0[int(np.argmin(np.abs(x1 - v))), mid]  # noqa: E731
    cores = [at(v) for v in (-3 * math.pi / 4, -math.pi / 4, math.pi / 4, 3 * math.pi / 4)]
    seps = [at(v) for v in (-math.pi / 2, 0.0, math.pi / 2)]
    assert max(cores) < 0.5 * min(seps), (cores, seps)


def test_paper2d_landing_cells_bit_exact():
    prob = W.paper2d()
    plan = Plan(prob)
    chi = oracle.chi(prob)
    for n in (0, 37, prob.n_steps - 1):
        cells, exitf = plan.export_cells(0, n)
        torch.cuda.synchronize()
        rc, rf = oracle.step_cells(prob, n, chi)
        assert int((cells.cpu().numpy() != rc).sum()) == 0
        assert int((exitf.cpu().numpy() != rf).sum()) == 0
    plan.close()


def test_paper2d_adjoint_matches_oracle():
    prob = W.paper2d()
    lam0 = W.region_mean_weights(prob)
    g_ref, lamN_ref = oracle.adjoint(prob, lam0)
    plan = Plan(prob, precision="f64", ckpt_every=16)
    g, lamN = plan.adjoint(torch.from_numpy(lam0.reshape(-1)))
    torch.cuda.synchronize()
    g = g[0].cpu().numpy()
    plan.close()
    rel = float(np.abs(g - g_ref).max() / np.abs(g_ref).max())
    lam_err = float(np.abs(lamN.cpu().numpy() - lamN_ref.reshape(-1)).max())
    print(f"paper2d grad {g} oracle {g_ref} rel {rel:.2e}, lamN {lam_err:.2e}")
    assert g.shape == (4,)
    assert rel <= 1e-10
    assert lam_err <= 1e-11 * max(1.0, float(np.abs(lamN_ref).max()))

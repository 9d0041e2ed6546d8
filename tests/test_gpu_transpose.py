"""The step operator A_n = Q Psi^n of Eq. (e34)-(e36) and its transpose,
applied to caller data through the C ABI hook fk_apply_step.

* Adjoint identity <A_n x, y> = <x, A_n^T y> (the transposed step is the
  reverse sweep's scatter): FP64 within 1e-13 of the sum of absolute terms.
* Both products element by element against the oracle's explicit dense rows
  of A_n (fko_assemble_row): FP64 within 1e-12, FP32 within 1e-5 (relative
  to the largest entry), on a disc case (landing points handled one by one),
  box cases (separable box form in 2D and the periodic 3D slab), and 1D.
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

from paper_2104_14561_amd import Plan  # noqa: E402


def _case(name):
    if name == "disc2d":
        return W.cell2d(nx=41, ny=21, n_steps=4, D=2e-3, gh_q=6)
    if name == "box2d":
        return W.Problem(axes=[W.uniform_axis(0, 1, 37), W.uniform_axis(0, 2, 29)],
                         coef_kind="const", coef=(0.4, -0.7), D=0.01, region_kind="box",
                         gh_q=5, dt=0.01, n_steps=3)
    if name == "abc3d":
        return W.abc3d(n=11, n_steps=3, dt=0.02, D=2e-3, gh_q=4)
    if name == "bm1d":
        return W.bm1d(n=41, n_steps=3, gh_q=8)
    raise KeyError(name)


def _representative(prob):
    """Node index each node stands for: periodic images map to the node they
    copy (its column of A_n carries the same unknown)."""
    idx = np.indices(prob.shape)
    for a, ax in enumerate(prob.axes):
        if ax.periodic:
            idx[a][idx[a] == ax.n - 1] = 0
    return np.ravel_multi_index(tuple(idx), prob.shape).reshape(-1)


def _fold(cols, rep):
    """Sum the columns of images into the columns of their originals."""
    out = np.zeros_like(cols)
    for f in range(cols.shape[0]):
        np.add.at(out[f], rep, cols[f])
    return out


def _oracle_matrix(prob, n):
    act = oracle.active_nodes(prob)
    rows = []
    for j in act:
        row, _ = oracle.assemble_row(prob, n, int(j))
        rows.append(row.reshape(-1))
    return act, np.array(rows)


@pytest.mark.parametrize("form", ["fused", "ell"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("name", ["disc2d", "box2d", "abc3d", "bm1d"])
def test_step_operator_and_transpose(name, prec, form):
    prob = _case(name)
    if form == "ell" and any(ax.periodic for ax in prob.axes):
        pytest.skip("the assembled form is built for non-periodic axes only")
    d, J = prob.d, prob.n_nodes
    rep = _representative(prob)
    rng = np.random.default_rng(11)
    x = rng.uniform(-1.0, 1.0, size=(d + 1, J))
    x = x[:, rep]                      # images hold their originals' values
    y = rng.uniform(-1.0, 1.0, size=J)
    n = prob.n_steps - 2
    act, A = _oracle_matrix(prob, n)
    Ax_ref = np.zeros(J)
    Ax_ref[act] = A @ x.reshape(-1)
    ym = np.zeros(J)
    ym[act] = y[act]
    ATy_ref = _fold((A.T @ y[act]).reshape(d + 1, J), rep)

    plan = Plan(prob, precision=prec, form=form, ckpt_every=1)
    Ax = plan.apply_step(n, torch.from_numpy(x.reshape(-1))).double().cpu().numpy()
    ATy = plan.apply_step(n, torch.from_numpy(y), transpose=True).double().cpu().numpy()
    torch.cuda.synchronize()
    plan.close()
    ATy_raw = ATy.reshape(d + 1, J)
    ATy = _fold(ATy_raw, rep)

    tol = 1e-12 if prec == "f64" else 1e-5
    e1 = float(np.abs(Ax - Ax_ref).max())
    e2 = float(np.abs(ATy - ATy_ref).max()) / max(1.0, float(np.abs(ATy_ref).max()))
    lhs = float(np.dot(Ax, ym))
    rhs = float(np.dot(x.reshape(-1), ATy_raw.reshape(-1)))
    scale = float(np.abs(Ax_ref * ym).sum()) + 1e-300
    gap = abs(lhs - rhs) / scale
    print(f"{name} {prec} {form}: |Ax - oracle| {e1:.2e}, |A^T y - oracle| {e2:.2e}, "
          f"dot gap {gap:.2e} (<Ax,y> = {lhs:.6e})")
    assert e1 <= tol
    assert e2 <= tol
    if prec == "f64":
        assert gap <= 1e-13


def test_transpose_needs_adjoint_plan():
    from paper_2104_14561_amd import FkError
    prob = _case("disc2d")
    plan = Plan(prob)
    with pytest.raises(FkError, match="FK_ERR_STATE"):
        plan.apply_step(0, torch.zeros(prob.n_nodes, dtype=torch.float64), transpose=True)
    with pytest.raises(FkError, match="FK_ERR_ARG"):
        plan.apply_step(prob.n_steps, torch.zeros(3 * prob.n_nodes, dtype=torch.float64))
    plan.close()

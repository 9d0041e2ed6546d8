"""Adjoint of the HIP path against the FP64 CPU oracle's adjoint (which is
itself pinned to central differences with frozen exit classification)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from bars import STATE_REL_DIFF, lamN_sensitivity
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import Plan  # noqa: E402
from paper_2104_14561_amd.autograd import exit_probability  # noqa: E402


def _lam0(prob, seed=21):
    rng = np.random.default_rng(seed)
    return rng.uniform(size=prob.shape)


def _gpu_adjoint(probs, lam0s, prec="f64", K=4, kernel="auto"):
    plan = Plan(probs, precision=prec, ckpt_every=K, step_kernel=kernel)
    lam = torch.cat([torch.from_numpy(l.reshape(-1)) for l in lam0s]).cuda()
    grad, lamN = plan.adjoint(lam)
    torch.cuda.synchronize()
    out = grad.cpu().numpy(), [x.double().cpu().numpy() for x in plan.split(lamN)]
    plan.close()
    return out


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("kernel", ["auto", "node", "box", "group"])
@pytest.mark.parametrize("case", ["cell2d", "const1d", "abc3d", "box2d"])
def test_adjoint_matches_oracle_fp64(case, kernel):
    if case == "cell2d":
        prob = W.cell2d(nx=65, ny=33, n_steps=14, dt=2e-3, D=2e-3, A=1.1, eps=0.2, omega=5.0)
    elif case == "box2d":
        # box exit: every node separable, footprints touching the faces
        prob = W.Problem(axes=[W.uniform_axis(0, 1, 37), W.uniform_axis(0, 2, 71)],
                         coef_kind="const", coef=(0.4, -0.7), D=0.01, region_kind="box",
                         gh_q=5, dt=0.01, n_steps=9)
    elif case == "const1d":
        prob = W.Problem(axes=[W.uniform_axis(-1, 1, 61)], coef_kind="const", coef=(0.3,),
                         D=0.2, region_kind="box", gh_q=6, dt=0.01, n_steps=15)
    else:
        prob = W.abc3d(n=13, n_steps=5, dt=0.05, D=3e-3)
    lam0 = _lam0(prob)
    g_ref, lamN_ref = oracle.adjoint(prob, lam0)
    gg, ll = _gpu_adjoint([prob], [lam0], kernel=kernel)
    g, lamN = gg[0], ll[0]
    nt = len(g_ref)
    print(case, g[:nt], g_ref, "lamN rel", _rel(lamN, lamN_ref))
    assert _rel(g[:nt], g_ref) <= 1e-10
    # lam^N passes through the PCHIP Jacobian of every u^n, whose derivative
    # depends on the ratio of divided differences: where rows are nearly flat
    # (the box case has translation-invariant rows) their rounding is
    # amplified.  The bar is the oracle's own change of lam^N per unit relative
    # perturbation of its states times the relative difference of the two
    # state sequences (and never below 1e-11)
    bar = max(1e-11, 4.0 * lamN_sensitivity(prob, lam0) * STATE_REL_DIFF)
    print(case, "lamN bar", bar)
    assert _rel(lamN, lamN_ref) <= bar


def test_checkpoint_interval_does_not_change_result():
    prob = W.cell2d(nx=49, ny=25, n_steps=13, dt=2e-3, D=3e-3)
    lam0 = _lam0(prob)
    ga, la = _gpu_adjoint([prob], [lam0], K=1)
    gb, lb = _gpu_adjoint([prob], [lam0], K=5)
    gc, lc = _gpu_adjoint([prob], [lam0], K=13)
    assert _rel(gb, ga) <= 1e-13 and _rel(gc, ga) <= 1e-13
    assert _rel(lb[0], la[0]) <= 1e-13 and _rel(lc[0], la[0]) <= 1e-13


def test_fp32_adjoint_close_to_fp64():
    prob = W.cell2d(nx=97, ny=49, n_steps=40, dt=1e-3, D=2e-3)
    cls = oracle.node_class(prob)
    lam0 = (cls == 0) / max((cls == 0).sum(), 1)      # mean of u^0 over the disc
    g64, _ = _gpu_adjoint([prob], [lam0], "f64", K=8)
    g32, _ = _gpu_adjoint([prob], [lam0], "f32", K=8)
    print(g64, g32)
    assert _rel(g32[0, :4], g64[0, :4]) <= 1e-3


def test_batched_adjoint_matches_single_instances():
    probs = W.cell2d_batch(n_inst=3, n_steps=8, max_m=2)
    lams = [_lam0(p, seed=30 + i) for i, p in enumerate(probs)]
    g, lN = _gpu_adjoint(probs, lams, "f64", K=3)
    for i, p in enumerate(probs):
        g_ref, l_ref = oracle.adjoint(p, lams[i])
        assert _rel(g[i, :4], g_ref) <= 1e-10
        assert _rel(lN[i], l_ref) <= 1e-11


def test_autograd_function_mean_over_disc():
    prob = W.cell2d(nx=49, ny=25, n_steps=10, dt=2e-3, D=3e-3)
    theta = torch.tensor([[1.0, 0.1, 6.0, 3e-3]], dtype=torch.float64, requires_grad=True)
    u0 = exit_probability(theta, [prob], "f64", 4)
    mask = torch.from_numpy((oracle.node_class(prob) == 0).reshape(-1)).cuda()
    J = (u0 * mask).sum() / mask.sum()
    J.backward()
    lam0 = (oracle.node_class(prob) == 0) / float(mask.sum())
    g_ref, _ = oracle.adjoint(prob.replace(coef=(1.0, 0.1, 6.0), D=3e-3), lam0)
    assert _rel(theta.grad.numpy()[0], g_ref) <= 1e-10


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_reuses_forward_checkpoints(prec):
    """fk_forward on a plan built for the adjoint stores the checkpoints; an
    adjoint on the same stream then skips its own forward pass.  Both routes,
    and an adjoint on another stream, give the same gradients up to the order
    of the atomic sums (the scatter and the gradient reduction add in
    scheduling order)."""
    tol = 1e-13 if prec == "f64" else 1e-5
    prob = W.cell2d(nx=65, ny=33, n_steps=21, dt=2e-3, D=2e-3)
    lam0 = torch.from_numpy(_lam0(prob).reshape(-1)).cuda()
    plan = Plan(prob, precision=prec, ckpt_every=4, use_graph=True)
    g_alone, l_alone = plan.adjoint(lam0)
    torch.cuda.synchronize()
    g_alone, l_alone = g_alone.cpu().numpy(), l_alone.cpu().numpy()
    plan.forward([0])
    g_reuse, l_reuse = plan.adjoint(lam0)
    torch.cuda.synchronize()
    assert _rel(g_reuse.cpu().numpy(), g_alone) <= tol
    assert _rel(l_reuse.cpu().numpy(), l_alone) <= tol
    side = torch.cuda.Stream()
    plan.forward([0])
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        g_side, _ = plan.adjoint(lam0, stream=side)
    torch.cuda.synchronize()
    assert _rel(g_side.cpu().numpy(), g_alone) <= tol
    plan.close()


def test_adjoint_matches_central_differences_of_gpu_forward():
    """Adjoint gradient against central differences (relative step h = 1e-6)
    of the GPU's own FP64 forward, the eight perturbed problems in one batched
    plan.  The scheme's J is piecewise smooth in theta: a landing point
    crossing the exit boundary switches its value to 1.  The oracle's exit
    records show that no landing point changes side within +-h here, so J is
    smooth over the difference stencil."""
    h = 1e-6
    prob = W.cell2d(nx=49, ny=25, n_steps=12, dt=2e-3, D=2e-3, A=1.1, eps=0.2, omega=5.0)
    theta = list(prob.coef) + [prob.D]
    _, rec = oracle.solve(prob, snaps=[0], record_exits=True)
    lam0 = _lam0(prob, seed=40)
    probs = []
    for k in range(len(theta)):
        for sgn in (1, -1):
            th = list(theta)
            th[k] = theta[k] * (1 + sgn * h)
            p = prob.replace(coef=tuple(th[:-1]), D=th[-1])
            _, r2 = oracle.solve(p, snaps=[0], record_exits=True)
            assert np.array_equal(r2, rec), "exit classification changes within the stencil"
            probs.append(p)
    (g,), _ = _gpu_adjoint([prob], [lam0], "f64", K=5)
    plan = Plan(probs, precision="f64", use_graph=True)
    out = plan.forward([0])
    J = [float(np.sum(lam0 * u.cpu().numpy())) for u in plan.split(out[0])]
    plan.close()
    fd = np.array([(J[2 * k] - J[2 * k + 1]) / (2 * h * abs(theta[k]))
                   for k in range(len(theta))])
    print("adjoint", g[:4], "central differences", fd)
    # the difference quotient's own error: rounding of J (per-node state
    # rounding ~1e-15, summed against lam0) over 2 h theta_k, plus O(h^2)
    fd_noise = 1e-15 * np.abs(lam0).sum() / (2 * h * np.abs(theta))
    assert np.all(np.abs(g[:4] - fd) <= 1e-5 * np.abs(fd) + fd_noise)

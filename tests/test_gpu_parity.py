"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: landing cells and exit flags bit-exact; FP64 fields within 1e-12 max
abs; FP32-apply fields (FP64 landing and cells) within 1e-5 max abs; the
assembled (ELL) form equal to the fused form within 1e-13 in FP64.
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

TOL = {"f64": 1e-12, "f32": 1e-5}


def _run(prob, prec="f64", snaps=(0,), **kw):
    plan = Plan(prob, precision=prec, **kw)
    out = plan.forward(list(snaps))
    torch.cuda.synchronize()
    assert plan.check_flags() == 0
    res = [r.double().cpu().numpy() for r in plan.split(out)]
    plan.close()
    return res


def _maxerr(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max())


# ---------------------------------------------------------------------------
# small cases: several tiles plus a ragged tail
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_bm1d_full(prec):
    prob = W.bm1d()
    snaps = [100, 60, 20, 0]
    ref = oracle.solve(prob, snaps=snaps)
    got = _run(prob, prec, snaps)[0]
    err = _maxerr(got, ref)
    print(f"bm1d {prec}: {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("kernel", ["node", "group", "split", "box"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(129, 65), (97, 53)])
def test_cell2d_small(prec, shape, kernel):
    prob = W.cell2d(nx=shape[0], ny=shape[1], n_steps=100, D=2e-3)
    snaps = [100, 50, 0]
    ref = oracle.solve(prob, snaps=snaps)
    got = _run(prob, prec, snaps, step_kernel=kernel)[0]
    err = _maxerr(got, ref)
    print(f"cell2d {shape} {prec} {kernel}: {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("kernel", ["node", "group", "split", "box"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abc3d_small(prec, kernel):
    prob = W.abc3d(n=21, n_steps=12, dt=0.02, D=2e-3)
    ref = oracle.solve(prob, snaps=[0, 6])
    got = _run(prob, prec, [0, 6], step_kernel=kernel)[0]
    err = _maxerr(got, ref)
    print(f"abc3d 21^3 {prec} {kernel}: {err:.3e}")
    assert err <= TOL[prec]


@pytest.mark.parametrize("kernel", ["node", "group", "split", "box"])
def test_box_exit_2d_and_ragged_q(kernel):
    """Box exit on both axes (separable exit mass), odd Q* and a grid that is
    not a multiple of any tile."""
    prob = W.Problem(axes=[W.uniform_axis(0, 1, 37), W.uniform_axis(0, 2, 71)],
                     coef_kind="const", coef=(0.4, -0.7), D=0.01, region_kind="box",
                     gh_q=5, dt=0.01, n_steps=25)
    ref = oracle.solve(prob, snaps=[0, 13])
    got = _run(prob, "f64", [0, 13], step_kernel=kernel)[0]
    assert _maxerr(got, ref) <= 1e-12


def test_const_drift_nonuniform_grid():
    rng = np.random.default_rng(5)
    x = np.sort(np.concatenate([[-1, 1], rng.uniform(-1, 1, 60)]))
    prob = W.Problem(axes=[W.Axis(x)], coef_kind="const", coef=(0.3,), D=0.05,
                     region_kind="box", gh_q=7, dt=0.01, n_steps=30)
    ref = oracle.solve(prob, snaps=[0])
    got = _run(prob, "f64", [0])[0]
    assert _maxerr(got, ref) <= 1e-12


@pytest.mark.parametrize("case", ["bm1d", "cell2d", "abc3d", "nonuniform2d"])
def test_landing_cells_bit_exact(case):
    if case == "bm1d":
        prob = W.bm1d()
        steps = [0, 99]
    elif case == "cell2d":
        prob = W.cell2d(nx=129, ny=65, n_steps=50)
        steps = [0, 17, 49]
    elif case == "abc3d":
        prob = W.abc3d(n=17, n_steps=5)
        steps = [0, 3]
    else:
        rng = np.random.default_rng(6)
        x = np.sort(np.concatenate([[0, 2], rng.uniform(0, 2, 70)]))
        y = np.sort(np.concatenate([[0, 1], rng.uniform(0, 1, 40)]))
        prob = W.cell2d(n_steps=10, D=4e-3).replace(axes=[W.Axis(x), W.Axis(y)])
        steps = [0, 9]
    plan = Plan(prob)
    u_dummy = oracle.chi(prob)
    for n in steps:
        cells, exitf = plan.export_cells(0, n)
        torch.cuda.synchronize()
        rc, rf = oracle.step_cells(prob, n, u_dummy)
        gf = exitf.cpu().numpy()
        gc = cells.cpu().numpy()
        mism_f = int((gf != rf).sum())
        mism_c = int((gc != rc).sum())
        print(f"{case} n={n}: exit-flag mismatches {mism_f}, cell mismatches {mism_c}")
        assert mism_f == 0 and mism_c == 0
    plan.close()


def test_single_step_from_random_state():
    prob = W.cell2d(nx=101, ny=61, n_steps=10, D=3e-3)
    u = W.random_field(prob.shape, seed=3)
    for n in (0, 7):
        ref = oracle.step(prob, n, u)
        plan = Plan(prob)
        got = plan.step(n, torch.from_numpy(u.reshape(-1)))
        torch.cuda.synchronize()
        got = got.double().cpu().numpy().reshape(prob.shape)
        assert _maxerr(got, ref) <= 1e-12
        plan.close()


# ---------------------------------------------------------------------------
# forms, graphs, batches, resume, determinism, flags
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ell_form_equals_fused(prec):
    prob = W.cell2d(nx=129, ny=65, n_steps=60, D=2e-3)
    a = _run(prob, prec, [0, 30], form="ell")[0]
    b = _run(prob, prec, [0, 30], form="fused")[0]
    ref = oracle.solve(prob, snaps=[0, 30])
    assert _maxerr(a, b) <= (1e-13 if prec == "f64" else 2e-6)
    assert _maxerr(a, ref) <= TOL[prec]


def test_ell_rows_match_oracle_rows():
    prob = W.cell2d(nx=65, ny=33, n_steps=4, D=4e-3, radius=0.4)
    plan = Plan(prob, form="ell")
    cols, vals, em = plan.export_ell(2)
    torch.cuda.synchronize()
    cols, vals, em = cols.cpu().numpy(), vals.cpu().numpy(), em.cpu().numpy()
    act = oracle.active_nodes(prob)
    J = prob.n_nodes
    for r in range(0, len(act), 37):
        row, emr = oracle.assemble_row(prob, 2, int(act[r]))
        dense = np.zeros(3 * J)
        np.add.at(dense, cols[:, r], vals[:, r])
        # oracle row is [field][node]; library columns are 3 * node + field
        ref = row.T.reshape(-1)
        assert np.abs(dense - ref).max() <= 1e-14
        assert abs(emr - em[r]) <= 1e-15
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", ["batch2d", "bm1d", "const3d"])
def test_ell_form_other_shapes(case, prec):
    """Assembled form on a batch of uneven grids (per-instance box widths,
    block padding and storage offsets), in 1D and in 3D."""
    if case == "batch2d":
        probs = W.cell2d_batch(n_inst=4, n_steps=10, max_m=3)
    elif case == "bm1d":
        probs = [W.bm1d(n=101, n_steps=20, gh_q=7)]
    else:
        probs = [W.Problem(axes=[W.uniform_axis(0, 1, 13), W.uniform_axis(0, 1, 11),
                                 W.uniform_axis(-1, 1, 17)],
                           coef_kind="const", coef=(0.3, -0.2, 0.1), D=4e-3, region_kind="box",
                           gh_q=3, dt=0.02, n_steps=6)]
    N = probs[0].n_steps
    a = _run(probs, prec, [0, N // 2], form="ell", use_graph=True)
    b = _run(probs, prec, [0, N // 2], form="fused", use_graph=True)
    for p, ga, gb in zip(probs, a, b):
        ref = oracle.solve(p, snaps=[0, N // 2])
        assert _maxerr(ga, gb) <= (1e-13 if prec == "f64" else 2e-6)
        assert _maxerr(ga, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_ell_export_batched_rows_match_oracle(prec):
    """fk_export_ell over two instances of different box widths: every
    sampled row of each instance equals the oracle's dense row of A_n."""
    probs = [W.cell2d(nx=65, ny=33, n_steps=4, D=4e-3, radius=0.4),
             W.cell2d(nx=97, ny=49, n_steps=4, D=1e-3, radius=0.35)]
    plan = Plan(probs, precision=prec, form="ell")
    cols, vals, em = plan.export_ell(2)
    torch.cuda.synchronize()
    cols, vals, em = cols.cpu().numpy(), vals.double().cpu().numpy(), em.double().cpu().numpy()
    tol = 1e-14 if prec == "f64" else 1e-6
    row0 = 0
    for i, prob in enumerate(probs):
        act = oracle.active_nodes(prob)
        J = prob.n_nodes
        base = plan.node_offset[i]
        for r in range(0, len(act), 41):
            row, emr = oracle.assemble_row(prob, 2, int(act[r]))
            dense = np.zeros(3 * J)
            c = cols[:, row0 + r] - 3 * base
            assert np.all((c >= 0) & (c < 3 * J))
            np.add.at(dense, c, vals[:, row0 + r])
            assert np.abs(dense - row.T.reshape(-1)).max() <= tol
            assert abs(emr - em[row0 + r]) <= tol
        row0 += len(act)
    plan.close()


def test_graph_replay_matches_eager():
    prob = W.cell2d(nx=97, ny=49, n_steps=40, D=2e-3)
    eager = _run(prob, "f64", [0, 20])[0]
    plan = Plan(prob, use_graph=True)
    outs = []
    for _ in range(3):
        o = plan.forward([0, 20])
        torch.cuda.synchronize()
        outs.append(plan.split(o)[0].cpu().numpy())
        _ = torch.ones(1000, device="cuda").sum().item()   # eager work between replays
    for o in outs:
        assert np.array_equal(o, eager)
    plan.close()


@pytest.mark.parametrize("kernel", ["auto", "box"])
def test_batched_uneven_grids_match_single_instances(kernel):
    probs = W.cell2d_batch(n_inst=5, n_steps=30, max_m=3)
    plan = Plan(probs, precision="f64", use_graph=True, step_kernel=kernel)
    out = plan.forward([0])
    torch.cuda.synchronize()
    parts = plan.split(out)
    for p, g in zip(probs, parts):
        ref = oracle.solve(p, snaps=[0])
        assert _maxerr(g.cpu().numpy(), ref) <= 1e-12
        single = _run(p, "f64", [0], step_kernel=kernel)[0]
        if kernel == "box":
            # same kernels in the single-instance plan: identical sums
            assert np.array_equal(g.cpu().numpy(), single)
        else:
            assert _maxerr(g.cpu().numpy(), single) <= 1e-13
    plan.close()


def test_resume_equals_uninterrupted():
    prob = W.cell2d(nx=81, ny=41, n_steps=30, D=2e-3)
    full = _run(prob, "f64", [0, 12])[0]
    plan = Plan(prob)
    mid = torch.from_numpy(full[1].reshape(-1)).cuda()
    res = plan.forward_from(mid, 12, [0])
    torch.cuda.synchronize()
    assert np.array_equal(plan.split(res)[0][0].cpu().numpy(), full[0])
    plan.close()


def test_deterministic_fp64():
    prob = W.abc3d(n=17, n_steps=6, D=2e-3)
    a = _run(prob, "f64", [0])[0]
    b = _run(prob, "f64", [0])[0]
    assert np.array_equal(a, b)


def test_nonfinite_state_is_flagged():
    prob = W.cell2d(nx=33, ny=17, n_steps=5, D=2e-3)
    plan = Plan(prob)
    u = torch.zeros(prob.n_nodes, dtype=torch.float64, device="cuda")
    # an active node at the disc centre (0.5, 0.5)
    u[8 * 17 + 8] = float("nan")
    plan.forward_from(u, 5, [0])
    torch.cuda.synchronize()
    from paper_2104_14561_amd.fkexit import FkError
    with pytest.raises(FkError) as ei:
        plan.check_flags()
    assert "NONFINITE" in str(ei.value)
    assert plan.check_flags() == 0     # cleared by the read
    plan.close()


# ---------------------------------------------------------------------------
# degenerate inputs and the largest rules
# ---------------------------------------------------------------------------

def _degenerate(case):
    b = W.cell2d(nx=33, ny=17, n_steps=6)
    if case == "empty_instance":
        # a disc that holds no node: every node exits, u = 1 throughout
        empty = W.cell2d(nx=33, ny=17, n_steps=6, radius=0.02, center=(0.53, 0.53))
        return [b, empty, b.replace(D=3e-3)]
    if case == "D0":        # sigma = 0: the Q landing points of a node coincide
        return [b.replace(D=0.0)]
    if case == "q1":        # one GH node at 0: the deterministic characteristic
        return [b.replace(gh_q=1)]
    if case == "one_step":
        return [b.replace(n_steps=1)]
    if case == "q64_1d":    # the largest rule, Q = 64
        return [W.bm1d(n=101, gh_q=64, n_steps=10)]
    if case == "q16_2d":    # Q = 256, the largest tensor rule
        return [b.replace(gh_q=16, n_steps=3)]
    if case == "q6_3d":     # Q = 216
        return [W.abc3d(n=9, n_steps=3, dt=0.05, D=3e-3)]
    raise ValueError(case)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", ["empty_instance", "D0", "q1", "one_step", "q64_1d",
                                  "q16_2d", "q6_3d"])
def test_degenerate_inputs(case, prec):
    probs = _degenerate(case)
    N = probs[0].n_steps
    snaps = sorted({N, N // 2, 0}, reverse=True)
    got = _run(probs, prec, snaps, use_graph=True)
    for p, g in zip(probs, got):
        ref = oracle.solve(p, snaps=snaps)
        err = _maxerr(g, ref)
        print(case, prec, p.gh_q, err)
        assert err <= TOL[prec]
        if oracle.active_nodes(p).size == 0:
            assert np.all(g == 1.0)


def test_degenerate_adjoint_with_empty_instance():
    """An instance without active nodes in a batched adjoint: zero gradient,
    zero lambda^N (exit nodes carry no cotangent), the others as alone."""
    probs = _degenerate("empty_instance")
    rng = np.random.default_rng(7)
    lams = [rng.uniform(size=p.shape) for p in probs]
    plan = Plan(probs, precision="f64", ckpt_every=4, use_graph=True)
    lam = torch.cat([torch.from_numpy(l.reshape(-1)) for l in lams]).cuda()
    g, lN = plan.adjoint(lam)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    lN = [x.cpu().numpy() for x in plan.split(lN)]
    plan.close()
    assert np.all(g[1] == 0.0) and np.all(lN[1] == 0.0)
    for i in (0, 2):
        g_ref, l_ref = oracle.adjoint(probs[i], lams[i])
        assert np.abs(g[i, :len(g_ref)] - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
        assert np.abs(lN[i] - l_ref).max() <= 1e-11 * np.abs(l_ref).max()


# ---------------------------------------------------------------------------
# full-size workloads
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_cell2d_full_size(prec):
    """513 x 257, disc target, 8x8 nodes, 1000 steps (oracle: ~30 s on 8 cores)."""
    prob = W.cell2d()
    ref = _cell2d_ref()
    got = _run(prob, prec, [1000, 500, 0], use_graph=True)[0]
    err = _maxerr(got, ref)
    print(f"cell2d full {prec}: {err:.3e}")
    assert err <= TOL[prec]


_REF = {}


def _cell2d_ref():
    if "cell2d" not in _REF:
        _REF["cell2d"] = oracle.solve(W.cell2d(), snaps=[1000, 500, 0])
    return _REF["cell2d"]


def test_autotuned_plan_matches_oracle():
    """fk_tune times the step layouts on this device; the plan built with its
    choice stays within the parity bar."""
    from paper_2104_14561_amd import tune
    probs = W.cell2d_batch(n_inst=3, n_steps=12, max_m=2)
    res = tune(probs, precision="f64", use_graph=True, trial_steps=4)
    print(res)
    assert res["step_kernel"] in ("node", "group", "split", "box")
    assert all(v > 0 for v in res["ms_per_step"].values())
    assert res["ms_per_step"][res["step_kernel"]] == min(res["ms_per_step"].values())
    plan = Plan(probs, precision="f64", use_graph=True, step_kernel="tune")
    assert plan.tuned is not None
    out = plan.forward([0])
    torch.cuda.synchronize()
    for p, g in zip(probs, plan.split(out)):
        assert _maxerr(g.cpu().numpy(), oracle.solve(p, snaps=[0])) <= 1e-12
    plan.close()

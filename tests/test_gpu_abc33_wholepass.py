"""Whole-pass parity of the 8-instance ABC-flow batch on 33^3 grids (6^3
Gauss-Hermite nodes, 500 steps: the benchmark batch's seeded D values at a
size the oracle finishes) against the FP64 oracle's stored values
(tests/golden/abc3d_33_oracle.json, written by make_abc3d_33.py, which calls
only the oracle).

Per instance, u^0 at the stored sample of active nodes and the sum of u^0 over
all active nodes; the gradient of J0 (mean of u^0 off the z faces) with
respect to (A, B, C, amp, D) for instance 0.

FP64 bar, derived as for the 2D batch: a step's value is a sum over Q = 216
tensor points of a weight times a 32-term Hermite value (8 corners x value and
three slopes), n ~ 256 operations deep with sum |terms| <= 3.25, so two
correct FP64 implementations differ per step by at most eps1 = 2e-13; the
oracle's measured response to per-step perturbations of delta = 1e-16 (random
r64, coherent rc) scaled by K = eps1 / delta = 2000, never below the stated
1e-12 nor above the stated FP32 bar 1e-5.  Gradient: K times the oracle's own
gradient change under the random perturbations, at least 1e-9 relative.

FP32 (the precision probe's instances in FP64, as the benchmark runs): 1e-5 on
u^0 plus the FP64 bar; the gradient within 1e-4 relative plus the FP64 bar.
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2104_14561_amd import Plan, precision_probe  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
FIXTURE = os.path.join(HERE, "golden", "abc3d_33_oracle.json")
EPS1 = 2e-13
K = EPS1 / 1e-16


def _fixture():
    if not os.path.exists(FIXTURE):
        pytest.skip("fixture not written (tests/golden/make_abc3d_33.py)")
    with open(FIXTURE) as fh:
        return json.load(fh)["instances"]


def _bar64(rec):
    return min(1e-5, max(1e-12, K * max(rec["r64"], rec["rc"])))


def _grad_bar64(rec):
    g = np.array(rec["grad"])
    return max(1e-9 * np.abs(g).max(), K * float(np.abs(np.array(rec["grad_p64"]) - g).max()))


def _lam0(probs):
    return torch.cat([torch.from_numpy(W.region_mean_weights(p).reshape(-1)) for p in probs])


def _run(probs, precision, force=None):
    plan = Plan(probs, precision=precision, use_graph=True, ckpt_every=1, force_f64=force)
    u0 = [t[0].double().cpu().numpy() for t in plan.split(plan.forward([0]))]
    g, _ = plan.adjoint(_lam0(probs))
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    plan.close()
    return u0, g


def _check(u0, g, probs, fx, extra, label):
    errs = []
    for i, (p, rec) in enumerate(zip(probs, fx)):
        u = u0[i].reshape(-1)
        idx = np.array(rec["index"])
        err = float(np.abs(u[idx] - np.array(rec["u0"])).max())
        bar = extra + _bar64(rec)
        errs.append((i, err, bar))
        act = oracle.active_nodes(p)
        s = float(u[act].sum())
        assert abs(s - rec["u0_active_sum"]) <= act.size * bar, (label, i, s, rec["u0_active_sum"])
    print(label, "u0 err/bar per instance:", " ".join(f"{i}:{e:.1e}/{b:.0e}" for i, e, b in errs))
    assert all(e <= b for _, e, b in errs), (label, errs)
    rec = fx[0]
    gr = np.array(rec["grad"])
    err = float(np.abs(g[0, :5] - gr).max())
    rel_extra = 1e-4 * float(np.abs(gr).max()) if extra > 0 else 0.0
    print(label, f"gradient rel err {err / np.abs(gr).max():.1e}")
    assert err <= rel_extra + _grad_bar64(rec), (label, g[0, :5], gr)


def test_abc33_fp64_whole_pass_matches_oracle():
    fx = _fixture()
    probs = W.abc3d_batch(n_inst=8, n=33)
    u0, g = _run(probs, "f64")
    _check(u0, g, probs, fx, 0.0, "FP64")


def test_abc33_fp32_with_probe_matches_oracle():
    fx = _fixture()
    probs = W.abc3d_batch(n_inst=8, n=33)
    force, _, _ = precision_probe(probs, tol=1e-5, lam0=_lam0(probs), grad_tol=1e-4, use_graph=True)
    u0, g = _run(probs, "f32", force)
    print("instances in FP64:", [i for i, f in enumerate(force) if f])
    _check(u0, g, probs, fx, 1e-5, "FP32+probe")

"""Writes abc3d_33_oracle.json: the FP64 CPU oracle's whole backward pass
(500 steps) of the 8-instance ABC-flow batch (the seeded D values of the
benchmark's 129^3 batch) on 33^3 grids, and the oracle's own sensitivity to
rounding there.

Every instance: u^0 at 256 seeded active nodes plus the node of each largest
response below, J0 (mean of u^0 over the nodes off the z faces), the sum of
u^0 over the active nodes, and
  * r64: the largest change of u^0 when every active value of every state u^n,
    n < N, receives an independent uniform perturbation in [-1e-16, 1e-16];
  * rc: the same when every such value is raised by 1e-16.
Instance 0 also carries the adjoint gradient of J0 with respect to
(A, B, C, amp, D) and grad_p64, the reverse sweep's gradient over the randomly
perturbed states.

Calls only the oracle (and the workload definitions); about 80 minutes on 8
cores:  python tests/golden/make_abc3d_33.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_SAMPLES = 256
SEED = 33500
DELTA64 = 1e-16


def perturbed_pass(op, prob, act_mask, mode, seed, keep_states=False):
    """u^0 (and, with keep_states, every state) of a pass whose every new
    state is perturbed on the active nodes: "abs" by DELTA64 * U[-1, 1],
    "coh" by +DELTA64."""
    rng = np.random.default_rng(seed)
    u = oracle.chi(op)
    U = None
    if keep_states:
        U = np.empty((prob.n_steps + 1,) + prob.shape)
        U[prob.n_steps] = u
    for n in range(prob.n_steps - 1, -1, -1):
        u = oracle.step(op, n, u)
        if mode == "abs":
            u = u + act_mask * (DELTA64 * rng.uniform(-1.0, 1.0, size=u.shape))
        else:
            u = u + DELTA64 * act_mask
        if keep_states:
            U[n] = u
    return u.reshape(-1), U


def main(path: str = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                  "abc3d_33_oracle.json")):
    probs = W.abc3d_batch(n_inst=8, n=33)
    out = {"workload": "abc3d_batch(n_inst=8, n=33): 33^3, 6^3 Gauss-Hermite nodes, dt 2e-3, 500 steps",
           "objective": "mean of u^0 over the nodes off the z faces",
           "delta64": DELTA64, "instances": []}
    t0 = time.time()
    for i, prob in enumerate(probs):
        op = oracle.OracleProblem(prob)
        act = oracle.active_nodes(op)
        lam0 = W.region_mean_weights(prob)
        u0 = oracle.solve(op, snaps=[0])[0].reshape(-1)
        rec = {"i": i, "shape": list(prob.shape), "D": prob.D,
               "J0": float(np.dot(lam0.reshape(-1), u0)),
               "u0_active_sum": float(u0[act].sum())}
        mask = np.zeros(prob.n_nodes)
        mask[act] = 1.0
        mask = mask.reshape(prob.shape)
        sens = []
        for mode, key in (("abs", "r64"), ("coh", "rc")):
            keep = (i == 0 and mode == "abs")
            up, U = perturbed_pass(op, prob, mask, mode, SEED + i, keep_states=keep)
            du = np.abs(up - u0)
            rec[key] = float(du.max())
            sens.append(int(np.argmax(du)))
            if keep:
                gp, _ = oracle.adjoint_states(op, U, lam0)
                rec["grad_p64"] = [float(g) for g in gp]
                del U
        if i == 0:
            grad, _ = oracle.adjoint(op, lam0)
            rec["grad"] = [float(g) for g in grad]
        rng = np.random.default_rng(SEED + 1000 + i)
        idx = np.unique(np.concatenate([rng.choice(act, min(N_SAMPLES, act.size), replace=False),
                                        np.array(sens, dtype=np.int64)])).astype(int)
        rec["index"] = idx.tolist()
        rec["u0"] = [float(u0[j]) for j in idx]
        out["instances"].append(rec)
        print(f"[{i}] D {prob.D:.3e} r64 {rec['r64']:.2e} rc {rec['rc']:.2e}" +
              (f" grad {rec['grad']}" if "grad" in rec else "") + f"  {time.time() - t0:.0f} s",
              flush=True)
        with open(path + ".partial", "w") as f:
            json.dump(out, f)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    if os.path.exists(path + ".partial"):
        os.remove(path + ".partial")
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main()

"""Writes cell2d_adj_oracle.json: the FP64 CPU oracle's adjoint of the
513x257 cellular-flow problem (dt = 5e-4, 2000 steps, 8x8 Gauss-Hermite
nodes), for J = mean of u^0 over the disc, and central differences of J with
relative step h = 1e-6 in each parameter (A, eps, omega, D), once with the
exit classification frozen at the base parameters and once recomputed.

Also lamN_fp32_emulation: the relative difference of the l1 norms of the
oracle's dJ/du^N over its exact states and over the same states as an FP32
implementation holds them (rounded to FP32, values below the FP32 underflow
threshold of the PCHIP slope's products zeroed; tests/bars.py), the scale of
the FP32 dJ/du^N deviation.

Calls only the oracle (and the workload definitions).  About 30 minutes on
8 cores:  python tests/golden/make_cell2d_adj.py   (--augment adds the
emulation to an existing file)
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

sys.path.insert(0, os.path.join(ROOT, "tests"))
from bars import lamN_fp32_emulation  # noqa: E402

H = 1e-6
N_SAMPLES = 256
SEED = 2104


def main(path: str = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                  "cell2d_adj_oracle.json")):
    prob = W.cell2d_adj()
    lam0 = W.region_mean_weights(prob)
    t0 = time.time()
    u0, rec = oracle.solve(prob, snaps=[0], record_exits=True)
    J0 = float(np.sum(lam0 * u0[0]))
    print(f"forward with exit record: {time.time() - t0:.0f} s", flush=True)
    grad, lamN = oracle.adjoint(prob, lam0)
    print(f"adjoint: {time.time() - t0:.0f} s  grad {grad}", flush=True)

    theta = list(prob.coef) + [prob.D]
    fd = {"frozen": [], "recomputed": []}
    for k in range(len(theta)):
        for kind in ("frozen", "recomputed"):
            J = []
            for sgn in (1, -1):
                th = list(theta)
                th[k] = theta[k] * (1 + sgn * H)
                u = oracle.solve(prob, snaps=[0], coef=th[:-1], D=th[-1],
                                 frozen_exits=rec if kind == "frozen" else None)[0]
                J.append(float(np.sum(lam0 * u)))
            fd[kind].append((J[0] - J[1]) / (2 * H * abs(theta[k])))
        print(f"theta[{k}]: adjoint {grad[k]!r} frozen {fd['frozen'][k]!r} "
              f"recomputed {fd['recomputed'][k]!r}  {time.time() - t0:.0f} s", flush=True)

    flat = lamN.reshape(-1)
    rng = np.random.default_rng(SEED)
    idx = np.unique(np.concatenate([
        rng.choice(flat.size, N_SAMPLES, replace=False),
        [int(np.argmax(np.abs(flat)))]])).astype(int)
    out = {
        "problem": {"nx": prob.shape[0], "ny": prob.shape[1], "dt": prob.dt,
                    "n_steps": prob.n_steps, "gh_q": prob.gh_q,
                    "coef": list(prob.coef), "D": prob.D},
        "objective": "mean of u^0 over the nodes strictly inside the disc",
        "h_relative": H,
        "J0": J0,
        "grad": [float(g) for g in grad],
        "fd_frozen_exits": fd["frozen"],
        "fd_recomputed_exits": fd["recomputed"],
        "lamN_l1": float(np.abs(flat).sum()),
        "lamN_max_abs": float(np.abs(flat).max()),
        "lamN_index": idx.tolist(),
        "lamN_value": [float(flat[i]) for i in idx],
        "lamN_fp32_emulation": lamN_fp32_emulation(prob, lam0)[1],
    }
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, flush=True)


def augment(path: str = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "cell2d_adj_oracle.json")):
    with open(path) as f:
        out = json.load(f)
    prob = W.cell2d_adj()
    out["lamN_fp32_emulation"] = lamN_fp32_emulation(prob, W.region_mean_weights(prob))[1]
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("lamN_fp32_emulation", out["lamN_fp32_emulation"], "wrote", path, flush=True)


if __name__ == "__main__":
    if "--augment" in sys.argv[1:]:
        augment()
    else:
        main()

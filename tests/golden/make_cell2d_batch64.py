"""Writes cell2d_batch64_oracle.json: the FP64 CPU oracle's whole backward
pass (1000 steps) of every instance of the 64-instance cellular-flow batch,
and, where the oracle's cost allows, the gradient of J = mean of u^0 over the
disc with respect to (A, eps, omega, D) and the scheme's own sensitivity to
rounding.

Every instance: u^0 at 128 seeded active nodes, J0 and the sum of u^0 over
the active nodes, and rc: the largest change of u^0 over the stored sample
when every active value of every state u^n, n < N, is raised by 1e-16 (a
coherent perturbation: rounding differences of two implementations share a
sign at neighbouring nodes, which fine grids do not average out).

Instances on grids up to 385 x 193 (m <= 3; the coarse, advection-dominated
instances whose scheme amplifies perturbations are among them):
  * r64: the largest change of u^0 (max abs) when every active value of every
    state u^n, n < N, receives an independent uniform perturbation in
    [-1e-16, 1e-16] (about half an ulp of 1: the size of the rounding
    differences of two correct FP64 implementations that sum in different
    orders), seed fixed; r32: the same when every state is rounded to FP32
    (the storage of an FP32 implementation); the node of each largest change
    is added to the sample;
  * the adjoint gradient; for m <= 2 also grad_p64 / grad_p32, the gradients
    of the oracle's reverse sweep over the two perturbed state sequences.
Two larger instances (513 x 257 and 1025 x 513) also carry the gradient.
Every instance with a gradient also carries grad_p64 and grad_pc, the
gradients of the reverse sweep over the randomly and the coherently perturbed
state sequences (--augment adds them where missing).

Calls only the oracle (and the workload definitions).  The oracle costs about
1.9 ms per active node and 1000 steps on 8 threads (the whole batch about
70 minutes forward), the adjoint about 3.3 times that; this script takes
about 210 minutes on 8 cores:  python tests/golden/make_cell2d_batch64.py
With --augment it reads the existing file and adds only the keys missing from
it (the oracle is deterministic: every node's sum runs on one thread in a fixed
order, so the stored u^0 is what a new pass computes).
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

N_SAMPLES = 128
SEED = 2104561
DELTA64 = 1e-16


def perturbed_states(op, prob, act_mask, mode, seed):
    """All states u^N .. u^0 of a pass whose every new state is perturbed
    (mode "abs": + DELTA64 * U[-1, 1] on active nodes; "f32": rounded to
    FP32); array [N + 1, J], entry n = u^n."""
    N = prob.n_steps
    rng = np.random.default_rng(seed)
    U = np.empty((N + 1, prob.n_nodes))
    u = oracle.chi(op)
    U[N] = u.reshape(-1)
    for n in range(N - 1, -1, -1):
        u = oracle.step(op, n, u)
        if mode == "abs":
            u = u + act_mask * (DELTA64 * rng.uniform(-1.0, 1.0, size=u.shape))
        elif mode == "coh":
            u = u + DELTA64 * act_mask
        else:
            u = u.astype(np.float32).astype(np.float64)
        U[n] = u.reshape(-1)
    return U


def coherent_u0(op, prob, act_mask):
    """u^0 of a pass whose every new state is raised by DELTA64 on the active
    nodes."""
    u = oracle.chi(op)
    for n in range(prob.n_steps - 1, -1, -1):
        u = oracle.step(op, n, u) + DELTA64 * act_mask
    return u.reshape(-1)


def add_rc(rec, op, prob, act):
    mask = np.zeros(prob.n_nodes)
    mask[act] = 1.0
    u = coherent_u0(op, prob, mask.reshape(prob.shape))
    idx = np.array(rec["index"])
    rec["rc"] = float(np.abs(u[idx] - np.array(rec["u0"])).max())


def add_grad_sens(rec, op, prob, act, i):
    """grad_p64 / grad_pc: the reverse sweep's gradient over the randomly
    (seed SEED + i, as for r64) and the coherently perturbed states."""
    mask = np.zeros(prob.n_nodes)
    mask[act] = 1.0
    mask = mask.reshape(prob.shape)
    lam0 = W.region_mean_weights(prob)
    for mode, key in (("abs", "grad_p64"), ("coh", "grad_pc")):
        if key in rec:
            continue
        U = perturbed_states(op, prob, mask, mode, SEED + i)
        gp, _ = oracle.adjoint_states(op, U.reshape((prob.n_steps + 1,) + prob.shape), lam0)
        rec[key] = [float(g) for g in gp]
        del U


def augment(path):
    with open(path) as fh:
        out = json.load(fh)
    probs = W.cell2d_batch()
    t0 = time.time()
    for i, (prob, rec) in enumerate(zip(probs, out["instances"])):
        need_rc = "rc" not in rec
        need_g = "grad" in rec and not ("grad_p64" in rec and "grad_pc" in rec)
        if not (need_rc or need_g):
            continue
        op = oracle.OracleProblem(prob)
        act = oracle.active_nodes(op)
        if need_rc:
            add_rc(rec, op, prob, act)
        if need_g:
            add_grad_sens(rec, op, prob, act, i)
        print(f"[{i:2d}] {prob.shape} rc {rec['rc']:.2e}" +
              (f" grad_p64 {rec['grad_p64']} grad_pc {rec['grad_pc']}" if need_g else "") +
              f"  {time.time() - t0:.0f} s", flush=True)
        with open(path + ".partial", "w") as f:
            json.dump(out, f)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    if os.path.exists(path + ".partial"):
        os.remove(path + ".partial")
    print("wrote", path, flush=True)


def main(path: str = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                  "cell2d_batch64_oracle.json")):
    probs = W.cell2d_batch()
    out = {"workload": "cell2d_batch64 (workloads.cell2d_batch())",
           "objective": "mean of u^0 over the nodes strictly inside the disc",
           "delta64": DELTA64, "instances": []}
    t0 = time.time()
    for i, prob in enumerate(probs):
        m = (prob.shape[0] - 1) // 128
        op = oracle.OracleProblem(prob)
        act = oracle.active_nodes(op)
        lam0 = W.region_mean_weights(prob)
        u0 = oracle.solve(op, snaps=[0])[0].reshape(-1)
        rec = {"i": i, "m": m, "shape": list(prob.shape),
               "J0": float(np.dot(lam0.reshape(-1), u0)),
               "u0_active_sum": float(u0[act].sum())}
        sens_nodes = []
        if m <= 3:
            mask = np.zeros(prob.n_nodes)
            mask[act] = 1.0
            mask = mask.reshape(prob.shape)
            for mode, key in (("abs", "64"), ("f32", "32")):
                U = perturbed_states(op, prob, mask, mode, SEED + i)
                du = np.abs(U[0] - u0)
                rec["r" + key] = float(du.max())
                sens_nodes.append(int(np.argmax(du)))
                if m <= 2:
                    gp, _ = oracle.adjoint_states(
                        op, U.reshape((prob.n_steps + 1,) + prob.shape), lam0)
                    rec["grad_p" + key] = [float(g) for g in gp]
                del U
        if m <= 3 or i in (5, 9):
            grad, _ = oracle.adjoint(op, lam0)
            rec["grad"] = [float(g) for g in grad]
        rng = np.random.default_rng(SEED + 1000 + i)
        idx = np.unique(np.concatenate([rng.choice(act, min(N_SAMPLES, act.size), replace=False),
                                        np.array(sens_nodes, dtype=np.int64)])).astype(int)
        rec["index"] = idx.tolist()
        rec["u0"] = [float(u0[j]) for j in idx]
        add_rc(rec, op, prob, act)
        if "grad" in rec:
            add_grad_sens(rec, op, prob, act, i)
        out["instances"].append(rec)
        print(f"[{i:2d}] {prob.shape} " + " ".join(
            f"{k} {rec[k]:.2e}" for k in ("r64", "r32", "rc") if k in rec) +
            (f" grad {np.array(rec['grad'])}" if "grad" in rec else "") +
            f"  {time.time() - t0:.0f} s", flush=True)
        with open(path + ".partial", "w") as f:
            json.dump(out, f)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    if os.path.exists(path + ".partial"):
        os.remove(path + ".partial")
    print("wrote", path, flush=True)


if __name__ == "__main__":
    if "--augment" in sys.argv[1:]:
        augment(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                             "cell2d_batch64_oracle.json"))
    else:
        main()

"""Throughput of the backward Feynman-Kac pass on one MI355X.

A bench step is one whole backward pass u^N -> u^0 (every time step of the
workload) over the workload's synthetic inputs, already resident in HBM.
value = active grid points x time steps per second (grid-point-steps/s).

Prints one JSON line (rank 0) with the roofline of the dominant kernel, timed
live with HIP events on the launch stream, and the CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def step_flops(d: int, q: int, f32: bool):
    """Algorithmic flops of one landing point of the fused step.

    FP64 in both precisions (classification): landing coordinate (mul + add),
    in-cell position (sub + div) and ball distance (sub, mul, add) per axis.
    Precision of the plan: cubic Hermite basis (value and slope pair, 10 per
    axis), the tensor contraction ((d+1) 2^d multiply-adds) and the weighted
    accumulation (2)."""
    f64 = 7 * d
    fp = 10 * d + 2 * (d + 1) * (1 << d) + 2
    if not f32:
        f64, fp = f64 + fp, 0
    return f64, fp


def fused_roofline(prob, plan, ms_step: float):
    d = prob.d
    Q = prob.gh_q ** d
    Ja = sum(plan.active_count)
    f64, f32 = step_flops(d, prob.gh_q, plan.precision == "f32")
    # FP32-equivalent flops: an FP64 flop costs two FP32 flops of issue rate
    eq = Ja * Q * (2 * f64 + f32)
    achieved = eq / (ms_step * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s (FP32-equivalent: FP64 flops count twice)",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": "k_step_fused", "launch_ms": round(ms_step, 5),
            "flops_per_landing_point": {"fp64": f64, "plan_precision": f32},
            "landing_points_per_launch": Ja * Q}


def cpu_baseline(prob, n_sample_steps: int):
    import oracle
    sample = prob.replace(n_steps=n_sample_steps)
    oracle.build(force=False)
    t0 = time.perf_counter()
    oracle.solve(sample, snaps=[0])
    dt = time.perf_counter() - t0
    Ja = oracle.active_nodes(sample).shape[0]
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": Ja * n_sample_steps / dt, "unit": "grid-point-steps/s", "cores": cores,
            "kind": "oracle", "seconds": round(dt, 2),
            "sample": f"{prob.name}: first {n_sample_steps} of {prob.n_steps} steps, "
                      f"FP64 C oracle, OpenMP over active nodes (steps are equal in cost)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--form", default="fused", choices=["fused", "ell"])
    ap.add_argument("--cpu-steps", type=int, default=300)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path shards by instance or by slab, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2104_14561_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    prob = W.cell2d()
    print(f"[bench] workload {prob.name} {prob.shape} N={prob.n_steps} "
          f"{args.precision} {args.form}", file=sys.stderr, flush=True)
    plan = Plan(prob, precision=args.precision, form=args.form, use_graph=True)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        plan.forward([0])
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.forward([0])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    assert plan.check_flags() == 0
    ms_step = ms_total / args.steps
    Ja = sum(plan.active_count)
    gp_steps = Ja * prob.n_steps
    value = gp_steps / (ms_step * 1e-3)
    print(f"[bench] {ms_step:.3f} ms per pass, {value:.4e} gp-steps/s", file=sys.stderr, flush=True)

    prof = plan.profile_pass()
    ms_kernel = prof["step_fused"][0] if args.form == "fused" else prof["ell_apply"][0]
    roof = fused_roofline(prob, plan, prof["step_fused"][0]) if args.form == "fused" else None
    plan.close()

    # plain FP64 single-instance path: same workload, launches without a graph
    plan64 = Plan(prob, precision="f64", use_graph=False)
    plan64.forward([0])
    torch.cuda.synchronize()
    e0.record(stream)
    plan64.forward([0])
    e1.record(stream)
    torch.cuda.synchronize()
    ms64 = e0.elapsed_time(e1)
    plan64.close()

    out = {
        "metric": "grid-point-steps/s (active nodes x time steps per second)",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 apply, f64 landing/cells" if args.precision == "f32" else "f64",
        "data": "synthetic (analytic cellular flow; no dataset)",
        "config": {"workload": f"{prob.name}: cellular flow 513x257, disc exit r=0.3, "
                               f"8x8 Gauss-Hermite, dt=1e-3, 1000 steps",
                   "form": args.form, "graph": True, "active_nodes": Ja},
        "kernels_ms": {k: v[0] for k, v in prof.items()},
        "f64_plain_gp_steps_per_s": gp_steps / (ms64 * 1e-3),
        "roofline": roof,
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

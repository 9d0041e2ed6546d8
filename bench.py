"""Throughput of the backward Feynman-Kac pass on one MI355X.

A bench step is one whole backward pass u^N -> u^0 (all 1000 time steps) over
the batched workload: 64 seeded cellular-flow instances on uneven grids
(129x65 .. 1025x513), 8x8 Gauss-Hermite nodes, dt = 1e-3, FP32 apply with FP64
landing points and cells, all instances in one plan whose step loop is
captured once in a HIP graph and replayed.  Inputs are resident in HBM before
the timed region.  value = active grid points x time steps per second, summed
over instances.

Reported beside it: the plain FP64 single-instance GPU path on the same 64
instances (one plan per instance, per-step launches, no graph), the max abs
difference of the FP32 batch from that FP64 path, per-kernel durations, the
roofline of the dominant kernel timed live with HIP events on its launch
stream, the assembled (ELL) form on the single 513x257 instance against the HBM
roofline, and the CPU oracle timed on a bounded sample.
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

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E (published)


def node_kernel_flops(d: int, qs: int):
    """Algorithmic flops of the thread-per-node step per active node.

    FP64 (classification): d*qs per-axis landing coordinates, each z = c + S a
    (2), ball distance (2), floor guess (2), exact fix-up (4), in-cell position
    (2) -> 12 per axis point; ball sum (d-1) per tensor point.
    Plan precision (apply): per tensor point the 2^d (d+1)-term Hermite
    contraction as multiply-adds (2 (d+1) 2^d), the value offsets (2^d) and the
    weighted accumulation (2); per axis point the Hermite basis (10)."""
    Q = qs ** d
    f64 = 12 * d * qs + (d - 1) * Q
    fp = Q * (2 * (d + 1) * (1 << d) + (1 << d) + 2) + 10 * d * qs
    return f64, fp


def alu_roofline(probs, plan, ms_kernel: float, kernel: str):
    d, qs = probs[0].d, probs[0].gh_q
    Ja = sum(plan.active_count)
    f64, f32 = node_kernel_flops(d, qs)
    if plan.precision == "f64":
        f64, f32 = f64 + f32, 0
    # FP32-equivalent flops: an FP64 flop takes two FP32 flops of issue rate
    eq = Ja * (2 * f64 + f32)
    achieved = eq / (ms_kernel * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": kernel, "launch_ms": round(ms_kernel, 5),
            "flops_per_active_node": {"fp64": f64, "fp32": f32,
                                      "note": "FP64 counted twice (half the FP32 issue rate)"},
            "active_nodes_per_launch": Ja}


def ell_roofline(plan, ms_apply: float):
    """Algorithmic bytes of one ELL product: per row W (col int32 + value)
    pairs, the exit mass, the gathered record entry per pair, the row's own
    record value and the output value."""
    s = 4 if plan.precision == "f32" else 8
    W_ = int(plan.info.ell_width)
    rows = int(plan.info.n_active)
    bytes_ = rows * (W_ * (4 + s) + s + W_ * s + s + s)
    achieved = bytes_ / (ms_apply * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": "k_ell_apply",
            "launch_ms": round(ms_apply, 5), "bytes_per_launch": bytes_, "ell_width": W_}


def cpu_baseline(probs, n_sample_steps: int):
    import oracle
    oracle.build(force=False)
    gp = 0
    t0 = time.perf_counter()
    for p in probs:
        sample = p.replace(n_steps=n_sample_steps)
        oracle.solve(sample, snaps=[0])
        gp += oracle.active_nodes(sample).shape[0] * n_sample_steps
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": gp / dt, "unit": "grid-point-steps/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 2),
            "sample": f"all {len(probs)} instances, first {n_sample_steps} of "
                      f"{probs[0].n_steps} steps (steps are equal in cost), FP64 C oracle, "
                      f"OpenMP over active nodes"}


def timed_passes(plan, k: int, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = None
    e0.record(stream)
    for _ in range(k):
        out = plan.forward([0])
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / k, out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline line only")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(sharding by instance is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2104_14561_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream()
    probs = W.cell2d_batch()
    N = probs[0].n_steps
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
    log(f"workload cell2d_batch64: {len(probs)} instances, N={N}, FP32 apply, graph")

    plan = Plan(probs, precision="f32", use_graph=True)
    Ja = sum(plan.active_count)
    for _ in range(args.warmup):
        plan.forward([0])
    torch.cuda.synchronize()
    ms_step, out32 = timed_passes(plan, args.steps, stream)
    assert plan.check_flags() == 0
    value = Ja * N / (ms_step * 1e-3)
    log(f"{ms_step:.2f} ms per pass, {value:.4e} gp-steps/s")

    prof = plan.profile_pass()
    kernels_ms = {k: v[0] for k, v in prof.items() if v[1]}
    roof = alu_roofline(probs, plan, prof["step_fused"][0], "k_step_node (fused step)")
    u32 = out32[0].double().cpu()
    plan.close()
    del plan, out32
    torch.cuda.empty_cache()

    result = {
        "metric": "grid-point-steps/s (active nodes x time steps per second, all instances)",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (apply; f64 landing points and cells)",
        "data": "synthetic: seeded analytic cellular flows, no dataset",
        "config": {"workload": "cell2d_batch64: 64 seeded cellular-flow instances, grids "
                               "(128m+1)x(64m+1) m~U{1..8}, disc exit r=0.3, 8x8 Gauss-Hermite, "
                               "dt=1e-3, 1000 steps, one plan, one captured HIP graph",
                   "instances": len(probs), "active_nodes": Ja, "time_steps": N},
        "kernels_ms": kernels_ms,
        "roofline": roof,
    }

    if not args.no_extra:
        # plain FP64 single-instance path: one plan per instance, no graph
        t_plain = 0.0
        err = 0.0
        u32_parts = []
        off = 0
        for p in probs:
            u32_parts.append(u32[off:off + p.n_nodes])
            off += p.n_nodes
        errs = []
        for i, p in enumerate(probs):
            pl = Plan(p, precision="f64", use_graph=False)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            o = pl.forward([0])
            e1.record(stream)
            torch.cuda.synchronize()
            t_plain += e0.elapsed_time(e1)
            errs.append(float((o[0].cpu() - u32_parts[i]).abs().max()))
            pl.close()
        plain_rate = Ja * N / (t_plain * 1e-3)
        errs = np.array(errs)
        result["f64_plain_single_instance"] = {
            "gp_steps_per_s": plain_rate, "ms_all_instances": t_plain,
            "speedup_of_batched_f32": value / plain_rate,
            "f32_vs_f64_max_abs_diff": {
                "max": float(errs.max()), "median": float(np.median(errs)),
                "instances_within_1e-5": int((errs <= 1e-5).sum()), "instances": len(errs),
                "note": "instances beyond 1e-5 are the coarse, advection-dominated ones whose "
                        "FP64 scheme amplifies any perturbation (see DESIGN.md, conditioning)"}}
        log(f"plain FP64: {plain_rate:.4e} gp-steps/s, speedup {value / plain_rate:.2f}, "
            f"f32 vs f64: max {errs.max():.2e} median {np.median(errs):.2e}")

        # batched FP32 adjoint of the mean of u^0 over each disc
        import oracle
        pa = Plan(probs, precision="f32", ckpt_every=64)
        lam = torch.zeros(pa.n_nodes, dtype=torch.float32, device="cuda")
        off = 0
        for p in probs:
            m = torch.from_numpy((oracle.node_class(p) == 0).reshape(-1).astype(np.float32))
            lam[off:off + p.n_nodes] = (m / m.sum()).cuda()
            off += p.n_nodes
        pa.adjoint(lam)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g, _ = pa.adjoint(lam)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_adj = e0.elapsed_time(e1)
        pa.close()
        result["adjoint_batched_f32"] = {
            "objective": "mean of u^0 over each instance's disc; gradient w.r.t. (A, eps, omega, D)",
            "ms_per_pass": ms_adj, "gp_steps_per_s": Ja * N / (ms_adj * 1e-3),
            "includes": "checkpointed forward (K = 64), segment recompute, transposed sweep",
            "fwd_plus_adj_gp_steps_per_s": Ja * N / ((ms_adj + ms_step) * 1e-3),
            "grad_instance0": [float(x) for x in g[0].cpu()]}
        log(f"adjoint: {ms_adj:.1f} ms per pass")

        # assembled ELL form on the single 513x257 instance (HBM roofline)
        single = W.cell2d()
        pe = Plan(single, precision="f32", form="ell", use_graph=True)
        pe.forward([0])
        torch.cuda.synchronize()
        ms_ell, _ = timed_passes(pe, 1, stream)
        pp = pe.profile_pass()
        result["ell_single_instance"] = {
            "workload": "cell2d 513x257, 1000 steps, FP32, assembled each step",
            "gp_steps_per_s": sum(pe.active_count) * single.n_steps / (ms_ell * 1e-3),
            "kernels_ms": {k: v[0] for k, v in pp.items() if v[1]},
            "roofline_ell_apply": ell_roofline(pe, pp["ell_apply"][0])}
        pe.close()

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(probs, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

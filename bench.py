"""Throughput of the backward Feynman-Kac pass and its adjoint on one MI355X.

A bench step is the whole hot path over the batched workload: one backward
pass u^N -> u^0 (all 1000 time steps) followed by one adjoint pass (the
gradient of each instance's disc-mean exit probability with respect to
(A, eps, omega, D), with u checkpointed every 64 steps and recomputed).  The
workload is 64 seeded cellular-flow instances on uneven grids (129x65 ..
1025x513), 8x8 Gauss-Hermite nodes, dt = 1e-3, FP32 apply with FP64 landing
points and cells, all instances in one plan (the forward step loop captured
once in a HIP graph and replayed).  Inputs are resident in HBM before the
timed region.  value = active grid points x time steps per second of
forward + adjoint, summed over instances.

Reported beside it: forward-only and adjoint-only rates; the plain FP64
single-instance GPU path on the same 64 instances (one plan per instance,
per-step launches, no graph) with the FP32-vs-FP64 differences of u^0 and of
the gradients; per-kernel durations; the roofline of the dominant kernel
timed live with HIP events on its launch stream; the assembled (ELL) form on
the single 513x257 instance against the HBM roofline; and the CPU oracle
(forward + adjoint) timed on a bounded sample.
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
# lane-level FP64 LDS atomic adds per second of the chip: 2048 workgroups x 256
# lanes of conflict-free ds_add_f64 ran at 1.62-1.95e12 on one MI355X (20-24 CU
# cycles per wave instruction); the best of those runs
LDS_F64_ATOMIC_PEAK = 1.95e12
CKPT_LIST = (1, 4, 16, 64)   # checkpoint intervals tried, smallest first
CKPT_MEM_FRACTION = 0.5       # of free HBM the plan's workspace may take


def step_kernel_flops(d: int, qs: int):
    """Algorithmic flops of the thread-per-node forward step per active node.

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


def adjoint_kernel_flops(d: int, qs: int):
    """Algorithmic flops of the thread-per-node adjoint step per active node (2D).

    FP64: the landing classification as in the forward step.  Plan precision,
    per tensor point: value and z-derivative Hermite bases of the inner axis
    (34), the interpolant gradient as two (d+1)-term contractions over the
    2^d corners (64), the weighted gradient sums (11) and the 2^d (d+1)
    transposed weights (17); per outer axis point the two bases (34).  The
    2^d (d+1) = 12 scatter adds per point run as FP64 LDS atomics and are not
    counted as flops."""
    Q = qs ** d
    f64 = 12 * d * qs + (d - 1) * Q
    fp = Q * (34 + 64 + 11 + 17) + 34 * qs
    return f64, fp


def alu_roofline(flops, n_nodes: int, ms_kernel: float, kernel: str, precision: str):
    f64, f32 = flops
    if precision == "f64":
        f64, f32 = f64 + f32, 0
    # FP32-equivalent flops: an FP64 flop takes two FP32 flops of issue rate
    eq = n_nodes * (2 * f64 + f32)
    achieved = eq / (ms_kernel * 1e-3) / 1e12
    return {"bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": None,
            "kernel": kernel, "launch_ms": round(ms_kernel, 5),
            "flops_per_active_node": {"fp64": f64, "fp32": f32,
                                      "note": "FP64 counted twice (half the FP32 issue rate)"},
            "active_nodes_per_launch": n_nodes}


def ell_roofline(plan, ms_apply: float):
    """Algorithmic bytes of one product of the stored operator: every stored
    value once (the rows are dense node boxes, their columns implicit in the
    box origin), per row the origin (3 int32), the exit mass, its own record
    value and the output value, and the node records the gathers read, each
    once (d+1 entries padded to the record stride, all nodes of the plan)."""
    s = 4 if plan.precision == "f32" else 8
    entries = int(plan.info.ell_entries)
    rows = int(plan.info.n_active)
    ps = 2 if plan.problems[0].d == 1 else 4
    bytes_ = entries * s + rows * (12 + 3 * s) + plan.n_nodes * ps * s
    achieved = bytes_ / (ms_apply * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None, "kernel": "k_ell_apply",
            "launch_ms": round(ms_apply, 5), "bytes_per_launch": bytes_, "ell_entries": entries,
            "rows": rows}


def kernel_sources_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("fk_device.h", "fk_node_inst.hip", "fk_launch.hip", "fk_internal.h", "fk_host.cpp"):
        with open(os.path.join(ROOT, "paper_2104_14561_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a 1 GiB copy)
    from the committed counter runs, while the kernel sources are unchanged."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_cell2d_batch64.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sources_sha256_16") != kernel_sources_hash() or kernel not in t["kernels"]:
        return None
    k = t["kernels"][kernel]
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def disc_mean_weights(probs, dtype, device):
    """lam0 = dJ/du^0 for J = mean of u^0 over each instance's disc nodes."""
    import torch
    parts = [torch.from_numpy(W.region_mean_weights(p).reshape(-1)) for p in probs]
    return torch.cat(parts).to(device=device, dtype=dtype)


def cpu_baseline(probs, n_sample_steps: int):
    import oracle
    oracle.build(force=False)
    gp = 0
    t0 = time.perf_counter()
    for p in probs:
        sample = p.replace(n_steps=n_sample_steps)
        oracle.solve(sample, snaps=[0])
        oracle.adjoint(sample, W.region_mean_weights(sample))
        gp += oracle.active_nodes(sample).shape[0] * n_sample_steps
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": gp / dt, "unit": "grid-point-steps/s", "cores": cores, "kind": "oracle",
            "seconds": round(dt, 2),
            "sample": f"all {len(probs)} instances, first {n_sample_steps} of {probs[0].n_steps} "
                      f"steps (steps are equal in cost), forward pass + adjoint (recomputing "
                      f"u in full), FP64 C oracle, OpenMP over active nodes"}


def event_time(fn, k: int, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    out = None
    e0.record(stream)
    for _ in range(k):
        out = fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / k, out


def ell_batched(probs, stream):
    """Assembled ELL form on the batch: a shortened pass (every step costs the
    same), its rate and the HBM roofline of the product."""
    import torch
    from paper_2104_14561_amd import Plan
    n_ell = 50
    pb = Plan([p.replace(n_steps=n_ell) for p in probs], precision="f32", form="ell",
              use_graph=True)
    Ja = sum(pb.active_count)
    pb.forward([0])
    torch.cuda.synchronize()
    ms_eb, _ = event_time(lambda: pb.forward([0]), 1, stream)
    ppb = pb.profile_pass()
    roof = ell_roofline(pb, ppb["ell_apply"][0])
    roof["traffic"] = measured_traffic("void k_ell_apply<float, 2>")
    out = {"workload": f"cell2d_batch64, first {n_ell} steps, FP32, A_n assembled each step "
                       "(one dense node box per row, per-instance width, values in 16-byte "
                       "blocks of box nodes per field)",
           "gp_steps_per_s": Ja * n_ell / (ms_eb * 1e-3),
           "kernels_ms": {k: v[0] for k, v in ppb.items() if v[1]},
           "roofline_ell_apply": roof}
    pb.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-steps", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="headline line only")
    ap.add_argument("--ell-only", action="store_true",
                    help="only the assembled (ELL) form on the batch, as its own JSON line")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 1 GiB device-to-device once (a kernel of known traffic "
                         "that scales the HBM byte counters of a profiled run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the instances are independent and would be sharded over GPUs by cost)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2104_14561_amd import Plan

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream()
    if args.copy_probe:
        n = 1 << 28   # 2^28 float32 = 1 GiB read + 1 GiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {n * 4} bytes read, {n * 4} bytes written", file=sys.stderr)
        del src, dst
        torch.cuda.empty_cache()
    probs = W.cell2d_batch()
    N = probs[0].n_steps
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
    if args.ell_only:
        print(json.dumps({"ell_batched": ell_batched(probs, stream)}), flush=True)
        return
    log(f"workload cell2d_batch64: {len(probs)} instances, N={N}, FP32 apply, forward + adjoint")

    # the smallest checkpoint interval whose storage fits half of free HBM
    # (every step stored: the adjoint recomputes nothing)
    free, _ = torch.cuda.mem_get_info()
    ckpt = CKPT_LIST[-1]
    for k in CKPT_LIST:
        probe = Plan(probs, precision="f32", use_graph=True, ckpt_every=k, allocate=False)
        need = int(probe.info.workspace_bytes)
        probe.close()
        if need <= CKPT_MEM_FRACTION * free:
            ckpt = k
            break
    log(f"checkpoint every {ckpt} step(s)")
    plan = Plan(probs, precision="f32", use_graph=True, ckpt_every=ckpt)
    Ja = sum(plan.active_count)
    lam0 = disc_mean_weights(probs, plan.dtype, plan.device)

    def one_step():
        u = plan.forward([0])
        g, _ = plan.adjoint(lam0)
        return u, g

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    ms_step, (out32, g32) = event_time(one_step, args.steps, stream)
    assert plan.check_flags() == 0
    value = Ja * N / (ms_step * 1e-3)
    log(f"{ms_step:.2f} ms per forward + adjoint, {value:.4e} gp-steps/s")

    ms_fwd, _ = event_time(lambda: plan.forward([0]), args.steps, stream)
    ms_adj, _ = event_time(lambda: plan.adjoint(lam0), max(1, args.steps // 2), stream)
    log(f"forward {ms_fwd:.2f} ms, adjoint {ms_adj:.2f} ms")

    prof_f = plan.profile_pass()
    prof_a = plan.profile_adjoint(lam0)
    kernels_ms = {"forward": {k: v[0] for k, v in prof_f.items() if v[1]},
                  "adjoint": {k: v[0] for k, v in prof_a.items() if v[1]}}
    d, qs = probs[0].d, probs[0].gh_q
    # per bench step: the fused forward step runs in the forward pass (whose
    # checkpoints the adjoint reuses) and once more per recomputed step of the
    # adjoint; the per-point transposed step once per step
    n_recomp = prof_a["recompute_step"][1]
    t_step_kernel = prof_f["step_fused"][0] * (N + n_recomp)
    t_adj_kernel = prof_a["adjoint_step"][0] * prof_a["adjoint_step"][1]
    n_point = int(plan.info.adj_point_nodes)
    if t_adj_kernel >= t_step_kernel:
        roof = alu_roofline(adjoint_kernel_flops(d, qs), n_point, prof_a["adjoint_step"][0],
                            "k_adjoint_node (transposed step, nodes handled per landing point)",
                            plan.precision)
        # its real limit: FP64 LDS atomic adds, 2^d (d+1) per inside landing point
        adds = n_point * qs ** d * (1 << d) * (d + 1)
        rate = adds / (prof_a["adjoint_step"][0] * 1e-3)
        roof["lds_fp64_atomic_adds"] = {
            "per_launch_upper_bound": adds, "achieved_per_s": rate,
            "probe_peak_per_s": LDS_F64_ATOMIC_PEAK, "frac": round(rate / LDS_F64_ATOMIC_PEAK, 4),
            "note": "lane-level ds_add_f64 rate; peak measured with a conflict-free probe kernel"}
        kname = "void k_adjoint_node<float, 2, 8, true>"
    else:
        roof = alu_roofline(step_kernel_flops(d, qs), Ja, prof_f["step_fused"][0],
                            "k_step_node (fused step)", plan.precision)
        kname = "void k_step_node<float, 2, 8, 1, true>"
    roof["traffic"] = measured_traffic(kname)
    roof["share_of_step"] = round(max(t_adj_kernel, t_step_kernel) / ms_step, 4)
    u32 = out32[0].double().cpu()
    g32 = g32.double().cpu().numpy()
    plan.close()
    del plan, out32
    torch.cuda.empty_cache()

    result = {
        "metric": "grid-point-steps/s of forward + adjoint (active nodes x time steps per second, "
                  "all instances)",
        "value": value,
        "unit": "grid-point-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: seeded analytic cellular flows, no dataset",
        "config": {"workload": "cell2d_batch64: 64 seeded cellular-flow instances, grids "
                               "(128m+1)x(64m+1) m~U{1..8}, disc exit r=0.3, 8x8 Gauss-Hermite, "
                               "dt=1e-3, 1000 steps, one plan; step = backward pass (captured HIP "
                               "graph) + adjoint of the disc-mean exit probability w.r.t. "
                               "(A, eps, omega, D); u checkpointed every ckpt_every steps (the "
                               "smallest of 1, 4, 16, 64 whose storage fits half of free HBM)",
                   "ckpt_every": ckpt,
                   "instances": len(probs), "active_nodes": Ja, "time_steps": N,
                   "precision": "FP32 weights and accumulation, FP64 landing points and cells"},
        "forward_only": {"ms_per_pass": ms_fwd, "gp_steps_per_s": Ja * N / (ms_fwd * 1e-3)},
        "adjoint_only": {"ms_per_pass": ms_adj, "gp_steps_per_s": Ja * N / (ms_adj * 1e-3),
                         "includes": "checkpointed forward, segment recompute, transposed sweep"},
        "kernels_ms": kernels_ms,
        "roofline": roof,
    }

    if not args.no_extra:
        # plain FP64 single-instance path: one plan per instance, no graph
        t_plain = 0.0
        off = 0
        errs, gerr = [], []
        for i, p in enumerate(probs):
            pl = Plan(p, precision="f64", use_graph=False, ckpt_every=64)
            lam_i = disc_mean_weights([p], pl.dtype, pl.device)
            torch.cuda.synchronize()
            t, (o, g) = event_time(lambda: (pl.forward([0]), pl.adjoint(lam_i)[0]), 1, stream)
            t_plain += t
            errs.append(float((o[0].cpu() - u32[off:off + p.n_nodes]).abs().max()))
            g64 = g.cpu().numpy()[0]
            gerr.append((float(np.abs(g32[i, :len(g64)] - g64).max()), float(np.abs(g64).max())))
            off += p.n_nodes
            pl.close()
        plain_rate = Ja * N / (t_plain * 1e-3)
        errs = np.array(errs)
        gabs = np.array([e for e, _ in gerr])
        big = [e / n for e, n in gerr if n >= 1e-3]
        result["f64_plain_single_instance"] = {
            "gp_steps_per_s": plain_rate, "ms_all_instances": t_plain,
            "speedup_of_batched_f32": value / plain_rate,
            "f32_vs_f64_u0_max_abs_diff": {
                "max": float(errs.max()), "median": float(np.median(errs)),
                "instances_within_1e-5": int((errs <= 1e-5).sum()), "instances": len(errs),
                "note": "instances beyond 1e-5 are the coarse, advection-dominated ones whose "
                        "FP64 scheme amplifies any perturbation (conditioning of the scheme)"},
            "f32_vs_f64_grad": {
                "max_abs_diff": float(gabs.max()), "median_abs_diff": float(np.median(gabs)),
                "rel_diff_where_norm_ge_1e-3": {"max": float(max(big)), "median": float(np.median(big)),
                                                "instances": len(big)},
                "note": "instances whose disc-mean exit probability barely moves (gradient "
                        "norm below 1e-3) are compared in absolute terms only"}}
        log(f"plain FP64: {plain_rate:.4e} gp-steps/s, speedup {value / plain_rate:.2f}, "
            f"u0 diff max {errs.max():.2e} median {np.median(errs):.2e}, "
            f"grad abs diff max {gabs.max():.2e}, rel (norm >= 1e-3) median {np.median(big):.2e}")

        result["ell_batched"] = ell_batched(probs, stream)
        log(f"ELL batched: {result['ell_batched']['gp_steps_per_s']:.4e} gp-steps/s, apply "
            f"{result['ell_batched']['roofline_ell_apply']['achieved']} GB/s")

        # assembled ELL form on the single 513x257 instance (HBM roofline)
        single = W.cell2d()
        pe = Plan(single, precision="f32", form="ell", use_graph=True)
        pe.forward([0])
        torch.cuda.synchronize()
        ms_ell, _ = event_time(lambda: pe.forward([0]), 1, stream)
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

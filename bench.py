"""Throughput of the backward Feynman-Kac pass and its adjoint on one MI355X.

A bench step is the whole hot path over the batched workload: one backward
pass u^N -> u^0 (all 1000 time steps) followed by one adjoint pass (the
gradient of each instance's disc-mean exit probability with respect to
(A, eps, omega, D)).  The workload is 64 seeded cellular-flow instances on
uneven grids (129x65 .. 1025x513), 8x8 Gauss-Hermite nodes, dt = 1e-3, all
in one plan (the step loop captured once in a HIP graph and replayed), FP32
apply with FP64 landing points and cells; the instances whose FP32 result
misses 1e-5 in u^0 or 1e-4 (relative) in the gradient are computed in FP64
inside the same plan (the precision probe runs each instance's pass and
adjoint once in FP64 and once in FP32 before the timed region).  u is
checkpointed every K steps, K the smallest of 1, 4, 16, 64 whose storage fits
half of free HBM (K = 1 on one MI355X: the forward pass stores every step and
the adjoint recomputes nothing).  Inputs are resident in HBM before the timed
region.  value = active grid points x time steps per second of forward +
adjoint, summed over instances.

Reported beside it: forward-only and adjoint-only rates; the same step at
K = 64 (segment recompute); the plain FP64 single-instance GPU path on the
same 64 instances (one plan per instance, per-step launches, no graph) at
K = 1 and K = 64 with the batch's differences of u^0 and of the gradients
against it; per-kernel durations; the roofline of the dominant kernel (the
survey's flop counts, the live LDS atomic peak of the device and the HBM
traffic of the committed counter runs); the 8-instance 129^3 ABC batch
(FP32 forward + adjoint with respect to D); the assembled (ELL) form on the
batch and on the single 513x257 instance against the HBM roofline;
Algorithm 1 (eight horizons of the 513x257 instance in one sweep); the host
and ROCm versions; and the CPU oracle (forward + adjoint) timed on a bounded
sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP32_TFLOPS = 157.3   # MI355X vector FP32 (published)
PEAK_FP64_TFLOPS = 78.6    # MI355X vector FP64 (published)
PEAK_HBM_GBS = 8000.0      # MI355X HBM3E (published)
CKPT_LIST = (1, 4, 16, 64)   # checkpoint intervals tried, smallest first
CKPT_MEM_FRACTION = 0.5       # of free HBM the plan's workspace may take
ACCURACY = 1e-5               # FP32 target against FP64 (max abs of u^0)
GRAD_ACCURACY = 1e-4          # and of the gradients (relative to their largest entry)
# Algorithmic flops per landing point of the fused forward step, from the
# hot-path scope estimate (FP64 classification, FP32 apply): 2D 22 + 56,
# 3D 35 + 160; the transposed step counts three times the forward.
SCOPE_FLOPS = {2: (22, 56), 3: (35, 160)}
ADJOINT_FACTOR = 3


def scope_roofline(d: int, Q: int, n_nodes: int, ms: float, factor: int, precision: str,
                   kernel: str):
    """ALU roofline of a fused kernel with the scope's counts: t_roof =
    nodes x Q x (f64 / P64 + f32 / P32); frac = t_roof / t; achieved in
    FP32-equivalent TFLOP/s (an FP64 flop costs two FP32 issue slots)."""
    f64, f32 = (c * factor for c in SCOPE_FLOPS[d])
    if precision == "f64":
        f64, f32 = f64 + f32, 0
    t_roof = n_nodes * Q * (f64 / (PEAK_FP64_TFLOPS * 1e12) + f32 / (PEAK_FP32_TFLOPS * 1e12))
    frac = t_roof / (ms * 1e-3)
    return {"bound": "alu", "achieved": round(frac * PEAK_FP32_TFLOPS, 3),
            "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": round(frac, 4),
            "traffic": None, "kernel": kernel, "launch_ms": round(ms, 5),
            "flops_per_landing_point": {"fp64": f64, "fp32": f32,
                                        "source": f"scope estimate x {factor}"},
            "landing_points_per_launch": n_nodes * Q}


def builder_adjoint_flops(d: int, qs: int):
    """This build's own count for the thread-per-node transposed step (2D),
    per active node: FP64 classification 12 d Q* + (d-1) Q; per tensor point
    in FP32 the value and z-derivative bases of the inner axis (34), the
    interpolant gradient (64), the weighted gradient sums (11) and the 2^d
    (d+1) transposed weights (17); per outer axis point the two bases (34).
    The 2^d (d+1) scatter adds per point run as FP64 LDS atomics."""
    Q = qs ** d
    return {"fp64": 12 * d * qs + (d - 1) * Q, "fp32": Q * (34 + 64 + 11 + 17) + 34 * qs}


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


def traffic_table():
    """Per-kernel HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled by a
    1 GiB copy) from the committed counter runs, while the kernel sources are
    unchanged; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_cell2d_batch64.json")
    try:
        with open(path) as fh:
            t = json.load(fh)
    except OSError:
        return None
    if t.get("kernel_sources_sha256_16") != kernel_sources_hash():
        return None
    return t["kernels"]


def measured_traffic(kernels):
    """Calibrated HBM bytes of one launch of each named kernel, summed (the
    kernels one timed group launches once each), or None."""
    t = traffic_table()
    if isinstance(kernels, str):
        kernels = [kernels]
    if not t or any(k not in t for k in kernels):
        return None
    return sum(t[k]["fetch_bytes_per_launch"] + t[k]["write_bytes_per_launch"] for k in kernels)


def disc_mean_weights(probs, dtype, device):
    """lam0 = dJ/du^0 for J = mean of u^0 over each instance's target nodes."""
    import torch
    parts = [torch.from_numpy(W.region_mean_weights(p).reshape(-1)) for p in probs]
    return torch.cat(parts).to(device=device, dtype=dtype)


def host_info():
    info = {"cpu_count": os.cpu_count(), "python": platform.python_version()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                info["cpu_model"] = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    for path in ("/opt/rocm/.info/version", "/opt/rocm/.info/version-dev"):
        try:
            with open(path) as fh:
                info["rocm"] = fh.read().strip()
                break
        except OSError:
            continue
    try:
        import torch
        info["torch"] = torch.__version__
        info["gpu"] = torch.cuda.get_device_name(0)
    except Exception:   # noqa: BLE001
        pass
    return info


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
    """Mean milliseconds of fn over k calls, HIP events on the launch stream."""
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


def pick_ckpt(probs, free_bytes, force):
    from paper_2104_14561_amd import Plan
    for k in CKPT_LIST:
        probe = Plan(probs, precision="f32", use_graph=True, ckpt_every=k, allocate=False,
                     force_f64=force)
        need = int(probe.info.workspace_bytes)
        probe.close()
        if need <= CKPT_MEM_FRACTION * free_bytes:
            return k
    return CKPT_LIST[-1]


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
    ms_asm = ppb["assemble_ell"][0]
    t = traffic_table()
    out = {"workload": f"cell2d_batch64, first {n_ell} steps, FP32, A_n assembled each step "
                       "(one dense node box per row, per-instance width, values in 16-byte "
                       "blocks of box nodes per field)",
           "gp_steps_per_s": Ja * n_ell / (ms_eb * 1e-3),
           "kernels_ms": {k: v[0] for k, v in ppb.items() if v[1]},
           "roofline_ell_apply": roof,
           "assembled_step_hbm": {
               "stored_value_bytes": int(pb.info.ell_entries) * 4,
               "ms_assembly_plus_product": round(ms_asm + ppb["ell_apply"][0], 4),
               "gbps_written_and_read": round(2 * int(pb.info.ell_entries) * 4
                                              / ((ms_asm + ppb["ell_apply"][0]) * 1e-3) / 1e9, 1),
               "note": "the values written by the assembly and read by the product, over the "
                       "two kernels' time"}}
    if t:
        out["traffic_per_launch"] = {k: v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"]
                                     for k, v in t.items() if "ell" in k}
    pb.close()
    return out


def abc3d_leg(stream, log):
    """The 8-instance 129^3 ABC batch: FP32 forward + adjoint with respect to
    D (and the flow amplitudes), every step stored."""
    import torch
    from paper_2104_14561_amd import Plan
    probs = W.abc3d_batch()
    N = probs[0].n_steps
    free, _ = torch.cuda.mem_get_info()
    ckpt = CKPT_LIST[-1]
    for k in CKPT_LIST:
        probe = Plan(probs, precision="f32", use_graph=True, ckpt_every=k, allocate=False)
        need = int(probe.info.workspace_bytes)
        probe.close()
        if need <= CKPT_MEM_FRACTION * free:
            ckpt = k
            break
    plan = Plan(probs, precision="f32", use_graph=True, ckpt_every=ckpt)
    Ja = sum(plan.active_count)
    lam0 = disc_mean_weights(probs, plan.dtype, plan.device)

    def step():
        u = plan.forward([0])
        g, _ = plan.adjoint(lam0)
        return u, g

    step()
    torch.cuda.synchronize()
    ms, (_, g) = event_time(step, 1, stream)
    ms_f, _ = event_time(lambda: plan.forward([0]), 1, stream)
    pf = plan.profile_pass()
    pa = plan.profile_adjoint(lam0)
    assert plan.check_flags() == 0
    dJdD = g[:, 4].double().cpu().tolist()
    plan.close()
    log(f"abc3d_batch8: {ms:.1f} ms per forward + adjoint, {Ja * N / (ms * 1e-3):.4e} gp-steps/s")
    return {"workload": "abc3d_batch8: 8 seeded D values, ABC flow (1, 0.8, 0.6)(1 + 0.1 sin t), "
                        "129^3 (x, y periodic, exit at |z| >= pi/2), 6x6x6 Gauss-Hermite, "
                        "dt = 2e-3, 500 steps, FP32 apply, adjoint of the mean of u^0 over the "
                        "active nodes",
            "ckpt_every": ckpt, "active_nodes": Ja, "ms_per_step": ms,
            "gp_steps_per_s": Ja * N / (ms * 1e-3),
            "forward_only": {"ms_per_pass": ms_f, "gp_steps_per_s": Ja * N / (ms_f * 1e-3)},
            "kernels_ms": {"forward": {k: v[0] for k, v in pf.items() if v[1]},
                           "adjoint": {k: v[0] for k, v in pa.items() if v[1]}},
            "dJ_dD": dJdD}


def algorithm1_leg(stream, log):
    """Algorithm 1 on the 513x257 cellular flow: eight horizons (125 .. 1000
    steps) in one backward sweep, FP32: the assembled operator applied to up
    to four columns per launch, the matrix-free step per column, and eight
    separate Scheme-1 passes."""
    import torch
    from paper_2104_14561_amd import Plan
    prob = W.cell2d()
    hz = [125 * (k + 1) for k in range(8)]
    out = {"workload": "cell2d 513x257, FP32, horizons 125, 250, .., 1000 steps",
           "column_steps": sum(hz)}
    for name, kw in (("ell_spmm_4col", {"form": "ell", "columns": 4}),
                     ("fused_per_column", {"form": "fused"})):
        pl = Plan(prob, precision="f32", use_graph=True, **kw)
        Ja = sum(pl.active_count)
        pl.forward_horizons(hz)
        torch.cuda.synchronize()
        ms, _ = event_time(lambda: pl.forward_horizons(hz), 1, stream)
        out[name] = {"ms": ms, "gp_steps_per_s": Ja * sum(hz) / (ms * 1e-3)}
        pl.close()
    ms_sep = 0.0
    for m in hz:
        pl = Plan(prob.replace(n_steps=m), precision="f32", use_graph=True)
        Ja = sum(pl.active_count)
        pl.forward([0])
        torch.cuda.synchronize()
        t, _ = event_time(lambda: pl.forward([0]), 1, stream)
        ms_sep += t
        pl.close()
    out["separate_scheme1_passes"] = {"ms": ms_sep, "gp_steps_per_s": Ja * sum(hz) / (ms_sep * 1e-3)}
    log(f"Algorithm 1: ELL SpMM {out['ell_spmm_4col']['ms']:.1f} ms, fused per column "
        f"{out['fused_per_column']['ms']:.1f} ms, separate passes {ms_sep:.1f} ms")
    return out


def extra_rows_leg(stream, log):
    """The forward pass of the extensions, each on its own workload: the
    paper's 2D roll-flow example (Section 4.2), the R2 interpolant against R1
    (2D cellular flow 513x257, 3D ABC flow 65^3), and the runaway-electron
    model (Section 4.3: exit-0 / exit-1 / reflecting faces, drift and
    diffusion per node, the non-uniform radial grid).  Whole-pass time and
    grid-point-steps/s, and the fused step's mean launch time."""
    import torch
    from paper_2104_14561_amd import Plan
    cases = [
        ("paper2d_rolls", W.paper2d(), {}, ("f64", "f32")),
        ("cell2d_513x257_r1", W.cell2d(), {}, ("f32",)),
        ("cell2d_513x257_r2", W.cell2d().replace(hermite="r2"), {"hermite": "r2"}, ("f32",)),
        ("abc3d_65_r1", W.abc3d(n=65, n_steps=100), {}, ("f32",)),
        ("abc3d_65_r2", W.abc3d(n=65, n_steps=100).replace(hermite="r2"),
         {"hermite": "r2", "step_kernel": "node"}, ("f32",)),
        ("runaway3d", W.runaway3d(), {}, ("f64", "f32")),
    ]
    out = {}
    for name, prob, kw, precs in cases:
        for prec in precs:
            pl = Plan(prob, precision=prec, use_graph=True, **kw)
            Ja = sum(pl.active_count)
            pl.forward([0])
            torch.cuda.synchronize()
            ms, _ = event_time(lambda: pl.forward([0]), 3, stream)
            prof = pl.profile_pass()
            pl.close()
            key = f"{name}_{prec}"
            out[key] = {"shape": list(prob.shape), "n_steps": prob.n_steps, "gh_q": prob.gh_q,
                        "active_nodes": Ja, "ms_per_pass": round(ms, 3),
                        "gp_steps_per_s": Ja * prob.n_steps / (ms * 1e-3),
                        "step_kernel_ms": round(prof["step_fused"][0], 5),
                        "slopes_ms": round(prof["slopes"][0], 5)}
            log(f"{key}: {ms:.2f} ms per pass, {out[key]['gp_steps_per_s']:.3e} gp-steps/s")
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
    ap.add_argument("--abc3d-only", action="store_true",
                    help="only the 129^3 ABC batch leg, as its own JSON line")
    ap.add_argument("--extensions-only", action="store_true",
                    help="only the forward passes of the extensions (roll flow, R2, runaway "
                         "model), as their own JSON line")
    ap.add_argument("--force-fp64", default=None,
                    help="comma-separated instances to compute in FP64 instead of running the "
                         "precision probe (profiling runs: the probe's selection given "
                         "explicitly, so that the profile holds only the timed kernels)")
    ap.add_argument("--no-profile", action="store_true",
                    help="skip the per-kernel profiling passes and the roofline (counter runs: "
                         "every kernel then runs in exactly two backward passes and two adjoints)")
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
    from paper_2104_14561_amd import Plan, precision_probe, probe_lds_atomics

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    stream = torch.cuda.current_stream()
    log = lambda *a: print("[bench]", *a, file=sys.stderr, flush=True)  # noqa: E731
    if args.copy_probe:
        n = 1 << 28   # 2^28 float32 = 1 GiB read + 1 GiB written
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy probe: {n * 4} bytes read, {n * 4} bytes written")
        del src, dst
        torch.cuda.empty_cache()
    probs = W.cell2d_batch()
    N = probs[0].n_steps
    if args.ell_only:
        print(json.dumps({"ell_batched": ell_batched(probs, stream)}), flush=True)
        return
    if args.abc3d_only:
        print(json.dumps({"abc3d_batch8": abc3d_leg(stream, log)}), flush=True)
        return
    if args.extensions_only:
        print(json.dumps({"extensions_forward": extra_rows_leg(stream, log)}), flush=True)
        return
    log(f"workload cell2d_batch64: {len(probs)} instances, N={N}, FP32 apply, forward + adjoint")

    # precision probe (before the timed region): instances whose FP32 u^0
    # misses the target run in FP64 inside the plan
    t0 = time.perf_counter()
    if args.force_fp64 is None:
        lam_probe = disc_mean_weights(probs, torch.float64, "cuda")
        force, pdiff, pgdiff = precision_probe(probs, tol=ACCURACY, lam0=lam_probe,
                                               grad_tol=GRAD_ACCURACY, use_graph=True)
        del lam_probe
    else:
        given = {int(v) for v in args.force_fp64.split(",") if v.strip()}
        force = [i in given for i in range(len(probs))]
        pdiff = pgdiff = None
    t_probe = time.perf_counter() - t0
    log(f"precision probe {t_probe:.1f} s: FP64 for instances {[i for i, f in enumerate(force) if f]}")

    free, _ = torch.cuda.mem_get_info()
    ckpt = pick_ckpt(probs, free, force)
    log(f"checkpoint every {ckpt} step(s)")
    plan = Plan(probs, precision="f32", use_graph=True, ckpt_every=ckpt, force_f64=force)
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

    if args.no_profile:
        print(json.dumps({"ms_per_step": ms_step, "forward_ms": ms_fwd, "adjoint_ms": ms_adj}),
              flush=True)
        return
    prof_f = plan.profile_pass()
    prof_a = plan.profile_adjoint(lam0)
    kernels_ms = {"forward": {k: v[0] for k, v in prof_f.items() if v[1]},
                  "adjoint": {k: v[0] for k, v in prof_a.items() if v[1]}}
    d, qs = probs[0].d, probs[0].gh_q
    Q = qs ** d
    n_recomp = prof_a["recompute_step"][1]
    t_step_kernel = prof_f["step_fused"][0] * (N + n_recomp)
    t_adj_kernel = prof_a["adjoint_step"][0] * prof_a["adjoint_step"][1]
    n_point = int(plan.info.adj_point_nodes)
    if t_adj_kernel >= t_step_kernel:
        ms_k = prof_a["adjoint_step"][0]
        roof = scope_roofline(d, Q, n_point, ms_k, ADJOINT_FACTOR, plan.precision,
                              "k_adjoint_node (transposed step, nodes handled per landing point)")
        bf = builder_adjoint_flops(d, qs)
        roof["builder_count"] = {
            "flops_per_active_node": bf,
            "frac": round(n_point * (2 * bf["fp64"] + bf["fp32"]) / (ms_k * 1e-3)
                          / (PEAK_FP32_TFLOPS * 1e12), 4)}
        # its ceiling on this device: FP64 LDS atomic adds, 2^d (d+1) per
        # inside landing point, against the rate measured live by the probe
        peak = probe_lds_atomics(f32=False)
        peak32 = probe_lds_atomics(f32=True)
        adds = n_point * Q * (1 << d) * (d + 1)
        rate = adds / (ms_k * 1e-3)
        roof["lds_fp64_atomic_adds"] = {
            "per_launch_upper_bound": adds, "achieved_per_s": rate, "probe_peak_per_s": peak,
            "probe_f32_adds_per_s": peak32,
            "frac": round(rate / peak, 4),
            "note": "lane-level ds_add_f64; peak from fk_probe_lds_atomics (2048 x 256 lanes, "
                    "conflict-free) on this device, this run"}
        # interior work items (no exit tests) and the rest: one launch each
        kname = ["void k_adjoint_node<float, 2, 8, true, true>",
                 "void k_adjoint_node<float, 2, 8, true, false>"]
        share = t_adj_kernel / ms_step
    else:
        ms_k = prof_f["step_fused"][0]
        roof = scope_roofline(d, Q, Ja, ms_k, 1, plan.precision, "k_step_node (fused step)")
        kname = "void k_step_node<float, 2, 8, 1, true, false, false>"
        share = t_step_kernel / ms_step
    roof["traffic"] = measured_traffic(kname)
    roof["share_of_step"] = round(share, 4)
    t = traffic_table()
    step_hbm = None
    if t:
        # HBM bytes of one bench step from the counter runs: every launch of
        # the forward pass and of the adjoint
        per = {k: v["fetch_bytes_per_launch"] + v["write_bytes_per_launch"] for k, v in t.items()}
        launches = {k: v.get("launches_per_step", 0) for k, v in t.items()}
        b = sum(per[k] * launches[k] for k in per)
        if b > 0:
            step_hbm = {"bytes_per_step": b, "gbps": round(b / (ms_step * 1e-3) / 1e9, 1),
                        "frac_of_peak": round(b / (ms_step * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    u32 = out32[0].double().cpu()
    g32 = g32.double().cpu().numpy()
    plan.close()
    del plan, out32
    torch.cuda.empty_cache()

    forced = [i for i, f in enumerate(force) if f]
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
                   "precision": "FP32 weights and accumulation, FP64 landing points and cells; "
                                "instances whose FP32 u^0 misses 1e-5 or whose FP32 gradient "
                                "misses 1e-4 relative in FP64",
                   "instances_in_fp64": forced},
        "precision_probe": {"seconds": round(t_probe, 2), "tol": ACCURACY,
                            "grad_tol": GRAD_ACCURACY, "instances_in_fp64": forced,
                            "f32_vs_f64_u0_max_abs": ([float(f"{x:.3g}") for x in pdiff]
                                                      if pdiff else "given by --force-fp64"),
                            "f32_vs_f64_grad_rel": ([float(f"{x:.3g}") for x in pgdiff]
                                                    if pgdiff else None)},
        "forward_only": {"ms_per_pass": ms_fwd, "gp_steps_per_s": Ja * N / (ms_fwd * 1e-3)},
        "adjoint_only": {"ms_per_pass": ms_adj, "gp_steps_per_s": Ja * N / (ms_adj * 1e-3),
                         "includes": ("transposed sweep over the checkpoints the forward pass "
                                      "stored (every step)" if ckpt == 1 else
                                      "segment recompute from the stored checkpoints, "
                                      "transposed sweep")},
        "kernels_ms": kernels_ms,
        "roofline": roof,
        "step_hbm": step_hbm,
        "host": host_info(),
    }

    if not args.no_extra:
        # the same batch at K = 64: the adjoint recomputes 63 of every 64 steps
        p64c = Plan(probs, precision="f32", use_graph=True, ckpt_every=64, force_f64=force)
        p64c.forward([0])
        p64c.adjoint(lam0)
        torch.cuda.synchronize()
        ms_k64, _ = event_time(lambda: (p64c.forward([0]), p64c.adjoint(lam0)), 1, stream)
        p64c.close()
        result["batch_ckpt_64"] = {"ms_per_step": ms_k64, "gp_steps_per_s": Ja * N / (ms_k64 * 1e-3)}
        log(f"batch at K=64: {ms_k64:.1f} ms")

        # plain FP64 single-instance path: one plan per instance, no graph, at
        # K = 1 (every step stored) and K = 64
        plain = {}
        errs, gerr = [], []
        for K in (1, 64):
            t_plain = 0.0
            off = 0
            for i, p in enumerate(probs):
                pl = Plan(p, precision="f64", use_graph=False, ckpt_every=K)
                lam_i = disc_mean_weights([p], pl.dtype, pl.device)
                pl.forward([0])
                torch.cuda.synchronize()
                t, (o, g) = event_time(lambda: (pl.forward([0]), pl.adjoint(lam_i)[0]), 1, stream)
                t_plain += t
                if K == 1:
                    errs.append(float((o[0].cpu() - u32[off:off + p.n_nodes]).abs().max()))
                    g64 = g.cpu().numpy()[0]
                    gerr.append((float(np.abs(g32[i, :len(g64)] - g64).max()),
                                 float(np.abs(g64).max())))
                off += p.n_nodes
                pl.close()
            plain[K] = t_plain
            log(f"plain FP64 K={K}: {t_plain:.1f} ms")
        errs = np.array(errs)
        gabs = np.array([e for e, _ in gerr])
        grel = np.array([e / n if n > 0 else (0.0 if e == 0 else np.inf) for e, n in gerr])
        big = [e / n for e, n in gerr if n >= 1e-3]
        result["f64_plain_single_instance"] = {
            "ckpt_1": {"ms_all_instances": plain[1], "gp_steps_per_s": Ja * N / (plain[1] * 1e-3),
                       "speedup_of_batched": plain[1] / ms_step},
            "ckpt_64": {"ms_all_instances": plain[64], "gp_steps_per_s": Ja * N / (plain[64] * 1e-3),
                        "speedup_of_batched_at_ckpt_64": plain[64] / ms_k64},
            "batched_vs_f64_u0_max_abs_diff": {
                "max": float(errs.max()), "median": float(np.median(errs)),
                "instances_within_1e-5": int((errs <= ACCURACY).sum()), "instances": len(errs)},
            "batched_vs_f64_grad": {
                "beyond_grad_tol": [
                    {"instance": i, "rel": float(f"{grel[i]:.3g}"),
                     "abs": float(f"{gerr[i][0]:.3g}"), "norm": float(f"{gerr[i][1]:.3g}"),
                     "in_fp64": bool(force[i])}
                    for i in range(len(grel)) if grel[i] > GRAD_ACCURACY],
                "max_abs_diff": float(gabs.max()), "max_rel_diff": float(grel.max()),
                "median_rel_diff": float(np.median(grel)),
                "rel_diff_where_norm_ge_1e-3": {"max": float(max(big)) if big else None,
                                                "instances": len(big)}},
            "note": "accuracy: the batched plan (FP32, probe-selected instances in FP64) "
                    "against the plain FP64 path; speed-ups at equal checkpoint interval"}
        log(f"batched vs plain FP64: u0 diff max {errs.max():.2e}, within 1e-5: "
            f"{int((errs <= ACCURACY).sum())}/{len(errs)}, grad rel max {grel.max():.2e}")

        result["abc3d_batch8"] = abc3d_leg(stream, log)
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
        result["algorithm1"] = algorithm1_leg(stream, log)
        result["extensions_forward"] = extra_rows_leg(stream, log)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(probs, args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

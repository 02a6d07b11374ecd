#!/usr/bin/env python3
"""Throughput of MPPI iterations on one MI355X.

A step is one pass of the whole hot path over one batch: `mppi_iterate(I)`
of the workload, i.e. I warm-started MPPI iterations, each made of noise
sampling, fused rollout + cost, and the softmin weighting + control update.
Default workload: the kinematic bicycle on a spline path with 200 circular
obstacles, K 8192 samples, horizon 100, 10 iterations per step.

Prints ONE JSON line with the throughput (rollout-steps/s = I*K*T / step time,
inputs resident in HBM), the roofline position of the dominant kernel measured
live with HIP events on the library's stream, and the binary64 CPU oracle timed
on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz; a wave64 VALU instruction
# issues over 4 cycles, so non-packed FP32 VALU lane-operations peak at
# 256 * 4 * 16 * 2.4e9 = 3.93e13 /s (78.6 TFLOP/s counting an FMA as 2).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_BYTES = 8.0e12
# Dense FP32 matrix-core peak of MI355X (v_mfma_f32_16x16x4_f32), FLOP/s.
MFMA_FP32_PEAK = 157.3e12


def mlp_macs(hidden: int) -> int:
    """Multiply-adds of one evaluation of the 7 -> H -> H -> 5 residual MLP."""
    return 7 * hidden + hidden * hidden + 5 * hidden

# Algorithmic VALU lane-operations per rollout step of the fused rollout +
# cost kernel (counted from the arithmetic the method needs; transcendental
# functions count as one operation each).  The derivation is in the design doc.
def rollout_ops_per_step(wl) -> int:
    v_form = wl.m                     # v = u + eps
    kahan = 4
    if wl.model == "bicycle":
        # RK4: 4 stages x (sin, cos, tan, 3 products, 1 scale) + 3 x 5 stage
        # updates + 3 x 5 accumulations + 5 final updates
        dyn = 4 * 7 + 15 + 15 + 5
    elif wl.model == "double_integrator":
        dyn = 4 if wl.integrator == "euler" else 4 * 4 + 40
    else:  # quadrotor: derivative ~ 60 ops, 4 stages + 3 x 13 stage updates + 13 x 4 accumulations + normalisation
        dyn = 4 * 60 + 39 + 52 + 9
    if wl.cost in ("path_circles", "path_costmap"):
        nseg = len(wl.knots) - 1
        cost = 2 + (nseg - 1) * 6 + 9 + 1 + 3 + 6 + 4 + 1  # clamp, select, cubic+slope, atan, errors, squares, controls, add
        if wl.cost == "path_circles":
            # crash test through the uniform obstacle grid: cell index (2 x
            # sub, mul, clamp x2, convert) + cell index + 2 list bounds, and
            # one candidate test (2 sub, mul, fma, compare) -- the useful work
            # of a point query, whatever the occupancy of its cell
            cost += 14 + 5
        else:
            cost += 20  # bilinear: index math, 4 gathers, 8 lerp ops
    elif wl.cost == "goal_circles":
        # goal distance (2 sub, mul, fma, scale), controls (2 mul, 2 fma),
        # grid crash query as for the path cost (14 + 5), crash add
        cost = 5 + 4 + 19 + 1
    elif wl.cost == "quadratic":
        cost = 3 * wl.n + 2 * wl.m
    elif wl.cost == "hover":
        cost = 40
    else:
        cost = 3 * wl.n + 2 * wl.m
    # the cost-complexity load: one operation per nested cosine
    return v_form + dyn + cost + kahan + int(getattr(wl, "cost_cosines", 0))


def make_workload(name: str):
    import workloads as W
    if name == "c2_circles":
        return W.c2("circles")
    if name == "c2_costmap":
        return W.c2("costmap")
    if name == "c1":
        return W.c1()
    if name == "c3":
        return W.c3()
    if name == "c4":
        return W.c4()
    if name == "c5":
        return W.c5()
    raise SystemExit(f"unknown workload {name}")


def source_hash(*rel):
    h = hashlib.sha256()
    for r in rel:
        with open(os.path.join(ROOT, r), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(kernel: str, workload: str, instance: str = ""):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source and on the kernel instance
    whose name contains `instance`; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash(*rec.get("sources", [])):
        return None
    if instance not in rec.get("kernel", ""):
        return None
    return rec.get("bytes_per_launch")


def phase_times(ctl, reps: int):
    """Average durations (s) of the sampling, rollout and update launches:
    HIP events recorded on the library's stream around `reps` back-to-back
    launches of each phase through the C ABI (so the dispatch latency of one
    launch is not counted)."""
    import torch
    import paper_2409_07563_amd as M
    L, ctx, stream = M.lib(), ctl.ctx, ctl.stream
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    out = []
    M._abi.check(L.mppi_sample(ctx))
    M._abi.check(L.mppi_rollout(ctx))
    for call in (L.mppi_sample, L.mppi_rollout, L.mppi_update):
        M._abi.check(call(ctx))  # warm
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            M._abi.check(call(ctx))
        ev[1].record(stream)
        torch.cuda.synchronize()
        out.append(ev[0].elapsed_time(ev[1]) / reps * 1e-3)
    return tuple(out)


def rollout_forms(tuned):
    """Fastest autotuned rollout launch (us) of the fused and of the split form."""
    if not tuned or "timings" not in tuned:
        return None
    best = {}
    for r in tuned["timings"]:
        if r["phase"] == "rollout":
            name = "split" if r.get("form") == 1 else "fused"
            best[name] = min(best.get(name, float("inf")), r["us"])
    return best or None


def copy_bandwidth(mib: int = 1024, reps: int = 10) -> float:
    """Achievable HBM bandwidth (GB/s, read + write bytes) of a device-to-device
    copy of `mib` MiB: the measured ceiling next to the 8 TB/s datasheet peak."""
    import torch
    a = torch.ones(mib << 18, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) / reps * 1e-3
    del a, b
    return 2.0 * (mib << 20) / s / 1e9


def cpu_baseline(wl, iters: int):
    import oracle
    t0 = time.perf_counter()
    oracle.mppi(wl, iters=iters)
    dt = time.perf_counter() - t0
    return {"value": iters * wl.K * wl.T / dt, "unit": "rollout-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{wl.name}: K {wl.K}, T {wl.T}, {iters} iterations "
                      f"(binary64 C oracle, single thread, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c2_circles")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle iterations for the CPU baseline (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of timing the candidates")
    ap.add_argument("--tuning", default=None,
                    help="launch shapes to apply instead of autotuning, as JSON "
                         "(e.g. the 'tuning' object of an earlier bench line)")
    ap.add_argument("--cost-cosines", type=int, default=0,
                    help="nested cosines ahead of every running cost (the cost-complexity "
                         "load of the paper's Results section)")
    ap.add_argument("--calibrate-copy-mb", type=int, default=0,
                    help="first run 3 device-to-device copies of this many MiB (a known "
                         "traffic reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2409_07563_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy_mb:
        n = args.calibrate_copy_mb << 18  # float32 elements
        a = torch.ones(n, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    wl = make_workload(args.workload)
    if args.cost_cosines:
        wl = ([w.replace(cost_cosines=args.cost_cosines) for w in wl] if isinstance(wl, list)
              else wl.replace(cost_cosines=args.cost_cosines))
    if isinstance(wl, list):
        return bench_batch(args, wl)
    if wl.model == "bicycle_mlp":
        return bench_grad(args, wl)
    I = wl.iters
    ctl = M.Controller(wl, device=dev)
    stream = ctl.stream
    tuned = None
    if args.tuning:
        ctl.set_tuning(**json.loads(args.tuning))
    elif not args.no_autotune:
        tuned = ctl.autotune(reps=30)

    for _ in range(args.warmup):
        ctl.iterate(I)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        ctl.iterate(I)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_per_step = start.elapsed_time(end) / args.steps
    steps_per_iter = wl.K * wl.T
    value = I * steps_per_iter / (ms_per_step * 1e-3)

    # the step with each form of the update that the context has
    update_forms = {}
    chosen = ctl.tuning()["update_form"]
    for form, name in ((0, "two_pass"), (1, "one_pass"), (2, "chunked")):
        try:
            ctl.set_tuning(update_form=form)
        except M.MPPIError:
            continue
        for _ in range(max(1, args.warmup)):
            ctl.iterate(I)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(args.steps):
            ctl.iterate(I)
        end.record(stream)
        torch.cuda.synchronize()
        update_forms[name] = start.elapsed_time(end) / args.steps
    ctl.set_tuning(update_form=chosen)

    t_noise, t_roll, t_upd = phase_times(ctl, args.kernel_reps)

    ops = rollout_ops_per_step(wl) * steps_per_iter
    achieved = ops / t_roll
    split = ctl.tuning()["rollout_form"] == 1
    lanes = ctl.tuning()["lanes_per_sample"]
    # the counters were taken on one kernel instance: the grouped kernel's
    # lane count is its last template argument
    traffic = traffic_record("rollout", args.workload,
                             f", {lanes}>" if lanes > 1 else "rollout_kernel<")
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS,
                "traffic": None if split else traffic,
                "kernel": ("split_dynamics + split_cost" if split else
                           "rollout_bicycle_group_kernel" if lanes > 1 else "rollout_kernel"),
                "ops_per_rollout_step": rollout_ops_per_step(wl), "launch_us": t_roll * 1e6}
    eps_bytes = 4 * wl.T * wl.m * wl.K
    kernels = {
        "noise": {"us": t_noise * 1e6, "hbm_GBps": eps_bytes / t_noise / 1e9},
        "rollout": {"us": t_roll * 1e6},
        "softmin_update": {"us": t_upd * 1e6, "hbm_GBps": (eps_bytes + 8 * wl.K) / t_upd / 1e9},
    }

    out = {
        "metric": "rollout-steps/sec (K*T) per MPPI iter + fwd+bwd/fwd time ratio, 1 MI355X",
        "value": value, "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "K": wl.K, "T": wl.T, "iterations_per_step": I,
                   "dynamics": wl.model, "integrator": wl.integrator, "cost": wl.cost,
                   "obstacles": 0 if wl.cx is None else len(wl.cx),
                   "cost_cosines": wl.cost_cosines},
        "fwd_bwd_over_fwd": None,
        "wall_s_timed": wall,
        "tuning": ctl.tuning(),
        "rollout_forms_us": rollout_forms(tuned),
        "update_forms_ms_per_step": update_forms,
        "roofline": roofline,
        "kernels": kernels,
        "achievable": {"hbm_copy_GBps": copy_bandwidth()},
    }
    ctl.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_iters or I)
    print(json.dumps(out), flush=True)


def bench_grad(args, wl):
    """Differentiable MPPI (MLP residual dynamics): the plain forward iteration,
    and one forward iteration in gradient mode (checkpointing rollout) plus the
    adjoint backward of L = |U - u_ref|^2, on the same GPU."""
    import numpy as np
    import torch
    import paper_2409_07563_amd as M
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    uref = torch.as_tensor(W.c5_uref(T=wl.T), device=dev)

    def timed(stream, fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps * 1e-3

    def measure(w):
        plain = M.Controller(w, device=dev)
        if not args.no_autotune:
            plain.autotune(reps=10)
        tuning = plain.tuning()
        t_fwd = timed(plain.stream, lambda: plain.iterate(1), args.steps, args.warmup)
        t_noise, t_roll, t_upd = phase_times(plain, args.kernel_reps)
        plain.close()
        grad = M.Controller(w, device=dev, requires_grad=True)
        # the same launch shapes as the plain forward (the gradient mode has
        # the two-pass update only: its adjoint reads the stored weights)
        grad.set_tuning(**{k: v for k, v in tuning.items() if k != "update_form"})
        grad.iterate(1)
        G = (2.0 * (grad.controls() - uref)).contiguous()
        L = M.lib()

        def fwd_bwd():
            M._abi.check(L.mppi_iterate(grad.ctx, 1))
            M._abi.check(L.mppi_backward(grad.ctx, G.data_ptr(), out.data_ptr()))
        out = torch.empty(grad.theta_len(), device=dev)
        grad._enter()
        t_fb = timed(grad.stream, fwd_bwd, args.steps, args.warmup)
        t_fg = timed(grad.stream, lambda: M._abi.check(L.mppi_iterate(grad.ctx, 1)),
                     args.steps, args.warmup)
        swept = int((grad.weights() > 0).sum())
        # three warm-started iterations and the reverse pass through all of
        # them (rebuilds each iteration from the tape, then its adjoint)
        du0 = torch.empty(wl.T * wl.m, device=dev)
        u0 = torch.as_tensor(w.u0, device=dev).contiguous()

        def fwd3():
            M._abi.check(L.mppi_set_controls(grad.ctx, u0.data_ptr()))
            M._abi.check(L.mppi_iterate(grad.ctx, 3))

        def fwd3_bwd():
            fwd3()
            M._abi.check(L.mppi_backward_iters(grad.ctx, G.data_ptr(), out.data_ptr(),
                                               du0.data_ptr()))
        t_f3 = timed(grad.stream, fwd3, args.steps, args.warmup)
        t_f3b = timed(grad.stream, fwd3_bwd, args.steps, args.warmup)
        grad.close()
        return t_fwd, t_noise, t_roll, t_upd, t_fb, t_fg, swept, tuning, t_f3, t_f3b

    t_fwd, t_noise, t_roll, t_upd, t_fb, t_fg, swept, tuning, t_f3, t_f3b = measure(wl)
    dense = wl.replace(lam=500.0)
    d_fwd, _, _, _, d_fb, d_fg, d_swept, _, _, _ = measure(dense)

    steps = wl.K * wl.T
    flops = 2.0 * mlp_macs(wl.mlp_hidden) * steps
    achieved = flops / t_roll
    eps_bytes = 4 * wl.T * wl.m * wl.K
    out = {
        "metric": "rollout-steps/sec (K*T) per MPPI iter + fwd+bwd/fwd time ratio, 1 MI355X",
        "value": steps / t_fwd, "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_fwd * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": wl.name, "K": wl.K, "T": wl.T, "iterations_per_step": 1,
                   "dynamics": wl.model, "hidden": wl.mlp_hidden, "integrator": wl.integrator,
                   "cost": wl.cost, "lambda": wl.lam, "checkpoint_every": 10},
        "fwd_bwd_over_fwd": (t_fb) / t_fwd,
        "tuning": tuning,
        "grad": {"fwd_plain_ms": t_fwd * 1e3, "fwd_checkpointing_ms": t_fg * 1e3,
                 "fwd_plus_bwd_ms": t_fb * 1e3, "bwd_ms": (t_fb - t_fg) * 1e3,
                 "samples_swept": swept,
                 "three_iterations": {"fwd_ms": t_f3 * 1e3, "fwd_plus_bwd_ms": t_f3b * 1e3,
                                      "fwd_bwd_over_fwd": t_f3b / t_f3},
                 "lambda_500": {"fwd_bwd_over_fwd": d_fb / d_fwd, "fwd_plus_bwd_ms": d_fb * 1e3,
                                "bwd_ms": (d_fb - d_fg) * 1e3, "samples_swept": d_swept}},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12,
                     "peak": MFMA_FP32_PEAK / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / MFMA_FP32_PEAK,
                     "traffic": traffic_record("rollout_tile", args.workload),
                     "kernel": "rollout_tile_kernel", "flops_per_rollout_step":
                         2 * mlp_macs(wl.mlp_hidden), "launch_us": t_roll * 1e6},
        "kernels": {"noise": {"us": t_noise * 1e6, "hbm_GBps": eps_bytes / t_noise / 1e9},
                    "rollout": {"us": t_roll * 1e6},
                    "softmin_update": {"us": t_upd * 1e6,
                                       "hbm_GBps": (eps_bytes + 8 * wl.K) / t_upd / 1e9}},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, 1)
    out["achievable"] = {"hbm_copy_GBps": copy_bandwidth()}
    print(json.dumps(out), flush=True)


def bench_batch(args, insts):
    """Many independent instances: one batched context (one launch per phase,
    the per-iteration sequence replayed from a hipGraph) against the same
    instances run one context after another on one stream."""
    import torch
    import paper_2409_07563_amd as M

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    total = sum(w.K * w.T for w in insts)
    ctl = M.Controller(insts, device=dev)
    stream = ctl.stream
    if not args.no_autotune:
        ctl.autotune(reps=3)
    tuning = ctl.tuning()

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    ms = timed(lambda: ctl.iterate(1), args.steps, args.warmup)
    tn, tr, tu = phase_times(ctl, max(1, args.kernel_reps // 5))
    ctl.close()

    # the same instances as single contexts, one after another on one stream
    # (each with the default launch shapes of its size)
    singles = [M.Controller(w, device=dev, stream=stream) for w in insts]
    def loop():
        for c in singles:
            c.iterate(1)
    ms_loop = timed(loop, max(1, args.steps // 4), 1)
    for c in singles:
        c.close()

    ops = sum(rollout_ops_per_step(w) * w.K * w.T for w in insts)
    achieved = ops / tr
    eps_bytes = sum(4 * w.T * w.m * w.K for w in insts)
    out = {
        "metric": "rollout-steps/sec (K*T) per MPPI iter + fwd+bwd/fwd time ratio, 1 MI355X",
        "value": total / (ms * 1e-3), "unit": "rollout-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "c4_batched_bicycle", "instances": len(insts),
                   "sum_K_T": total, "K_range": [min(w.K for w in insts), max(w.K for w in insts)],
                   "T_range": [min(w.T for w in insts), max(w.T for w in insts)],
                   "iterations_per_step": 1, "cost": insts[0].cost},
        "tuning": tuning,
        "looped_single_contexts": {"ms_per_step": ms_loop, "value": total / (ms_loop * 1e-3),
                                   "speedup_of_batch": ms_loop / ms},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": traffic_record("rollout", args.workload),
                     "kernel": "batch_rollout_kernel", "launch_us": tr * 1e6},
        "kernels": {"noise": {"us": tn * 1e6, "hbm_GBps": eps_bytes / tn / 1e9},
                    "rollout": {"us": tr * 1e6},
                    "softmin_update": {"us": tu * 1e6, "hbm_GBps": eps_bytes / tu / 1e9}},
    }
    out["achievable"] = {"hbm_copy_GBps": copy_bandwidth()}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Throughput of MPPI iterations on one MI355X.

A step is one pass of the whole hot path over one batch of synthetic input:
one warm-started MPPI iteration of every instance (noise sampling, fused
rollout + cost, the softmin weighting and the control update).  The default
run measures, on one GPU:

  * the headline: 256 independent bicycle instances (K 1024..16384, T 50..200,
    50..300 circular obstacles each) advanced by one batched context, one
    iteration per step; value = sum_i K_i T_i / step time (rollout-steps/s);
  * legs on the same GPU: the 13-state quadrotor at K 65536, T 200; the
    path-tracking bicycle with 200 obstacles at K 8192, T 100 (10 iterations
    per step); the bicycle with the MLP residual at K 8192, T 100, whose
    forward + adjoint backward time over the forward time is the metric's
    second half (fwd_bwd_over_fwd);
  * measured ceilings beside the datasheet peaks: the VALU issue rate of
    independent FMA (and exp, 64-bit multiply-add) chains, the HBM copy
    bandwidth, the launch floor of a captured graph and the latency of one
    wave's 100-step rollout chain;
  * the binary64 oracle on the host: one thread, and all the threads this
    process may use (instances spread over threads), with the CPU model.

Prints ONE JSON line.  Inputs are resident in HBM when a timed region
starts; every time comes from HIP events recorded on the stream the kernels
run on.  `--workload NAME` measures one workload on its own (the form the
profiler runs use).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout-steps/sec (K*T) per MPPI iter + fwd+bwd/fwd time ratio, 1 MI355X"
# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz.  A wave64 VALU instruction
# issues over 4 cycles on a 16-lane SIMD, so non-packed binary32 VALU
# lane-operations peak at 256 * 4 * 16 * 2.4e9 = 3.93e13 /s (78.6 TFLOP/s
# counting an FMA as 2; the 157.3 TFLOP/s vector figure needs packed FP32,
# which this build does not emit).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9
HBM_PEAK_BYTES = 8.0e12
# Dense FP32 matrix-core peak of MI355X (v_mfma_f32_16x16x4_f32), FLOP/s.
MFMA_FP32_PEAK = 157.3e12
# Dense BF16 matrix-core peak of MI355X, FLOP/s.
MFMA_BF16_PEAK = 2.5e15


def mlp_macs(hidden: int) -> int:
    """Multiply-adds of one evaluation of the 7 -> H -> H -> 5 residual MLP."""
    return 7 * hidden + hidden * hidden + 5 * hidden


def rollout_ops_per_step(wl) -> int:
    """Algorithmic VALU lane-operations of one rollout step (dynamics step +
    running cost + v = u + eps + the compensated cost sum), counted from the
    arithmetic the model and cost need: a fused multiply-add is one
    operation, a transcendental function one, sign and absolute-value source
    modifiers and exact power-of-two scalings are free, and terms that do not
    change over the four RK4 stages (the control held over the step) are
    formed once per step."""
    v_form = wl.m                     # v = u + eps
    kahan = 4
    if wl.model == "bicycle":
        # RK4: 4 stages x (sin, cos, tan, 3 products, 1 scale) + 3 x 5 stage
        # updates + 3 x 5 accumulations + 5 final updates
        dyn = 4 * 7 + 15 + 15 + 5
    elif wl.model == "double_integrator":
        dyn = 4 if wl.integrator == "euler" else 4 * 4 + 40
    else:
        # quadrotor: per stage q' 4 x 3, v' 3 x 3, omega' 3 x 2 (= 27), plus 6
        # per step (thrust / mass, its double, minus g, tau_j / J_j); RK4
        # combination 13 x 7; quaternion renormalisation 9
        dyn = 4 * 27 + 6 + 13 * 7 + 9
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
        # position error 3 + three squared norms 9 + attitude 4 + combination
        # 5; control error 8; box penalty 9; 2 adds
        cost = 40
    else:
        cost = 3 * wl.n + 2 * wl.m
    # the cost-complexity load: one operation per nested cosine
    return v_form + dyn + cost + kahan + int(getattr(wl, "cost_cosines", 0))


def make_workload(name: str):
    import workloads as W
    table = {"c2_circles": lambda: W.c2("circles"), "c2_costmap": lambda: W.c2("costmap"),
             "c1": W.c1, "c3": W.c3, "c4": W.c4, "c5": W.c5}
    if name not in table:
        raise SystemExit(f"unknown workload {name}")
    return table[name]()


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


def timed(stream, fn, steps: int, warmup: int) -> float:
    """Seconds per call of fn: `warmup` untimed calls, then HIP events on
    `stream` around exactly `steps` calls, synchronised on both sides."""
    import torch
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
    """Fastest autotuned rollout launch (us) of the fused, split and scan forms."""
    if not tuned or "timings" not in tuned:
        return None
    best = {}
    for r in tuned["timings"]:
        if r["phase"] == "rollout":
            name = {1: "split", 2: "scan"}.get(r.get("form"), "fused")
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


def measure_ceilings() -> dict:
    """Measured ceilings of this GPU (paper_2409_07563_amd.ceilings)."""
    import torch
    from paper_2409_07563_amd import ceilings as CE
    s = torch.cuda.Stream()
    valu = {}
    for mode in ("fma", "fma+exp", "exp", "mad_u64", "int_xor_add"):
        rate, _ = CE.valu(mode, blocks=16384, iters=1024, reps=5, stream=s)
        valu[mode] = rate
    return {
        "valu_lane_ops_per_s": valu,
        "valu_peak_derived": VALU_PEAK_OPS,
        "valu_fma_over_derived": valu["fma"] / VALU_PEAK_OPS,
        "hbm_copy_GBps": copy_bandwidth(),
        "graph_launch_us": {"3_kernels": CE.graph(3, 1, stream=s),
                            "3_kernels_x10_per_iteration": CE.graph(3, 10, stream=s) / 10},
        "chain_us": {f"T{T}": CE.chain(T, stream=s) for T in (50, 100, 200)},
    }


def host_info() -> dict:
    from oracle import oracle as O
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "threads_usable": O.host_threads(), "cpu_model": model}


# ---------------------------------------------------------------------------
# the oracle on the host (the CPU baseline)
# ---------------------------------------------------------------------------
def oracle_instances(insts, threads: int) -> float:
    """Seconds for one oracle iteration (noise, rollouts, update) of every
    instance, the instances spread over `threads` host threads (each call is
    the unmodified binary64 oracle; ctypes releases the interpreter lock)."""
    from oracle import oracle as O
    todo = list(range(len(insts)))[::-1]
    lock = threading.Lock()
    errors = []

    def work():
        while True:
            with lock:
                if not todo:
                    return
                i = todo.pop()
            try:
                O.mppi(insts[i], iters=1)
            except Exception as e:  # noqa: BLE001
                errors.append(e)
    ts = [threading.Thread(target=work) for _ in range(max(1, threads))]
    t0 = time.perf_counter()
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    dt = time.perf_counter() - t0
    if errors:
        raise errors[0]
    return dt


def cpu_baseline_batch(insts, n_single: int, n_all: int) -> dict:
    from oracle import oracle as O
    thr = O.host_threads()
    one = insts[:n_single]
    t1 = oracle_instances(one, 1)
    v1 = sum(w.K * w.T for w in one) / t1
    many = insts[:n_all]
    tn = oracle_instances(many, thr)
    vn = sum(w.K * w.T for w in many) / tn
    info = host_info()
    return {"value": vn, "unit": "rollout-steps/s", "cores": thr, "kind": "oracle",
            "sample": f"the first {n_all} of the 256 batched instances, one iteration each "
                      f"({sum(w.K * w.T for w in many):.3g} rollout-steps; binary64 C oracle, "
                      f"instances spread over {thr} threads, {tn:.1f} s)",
            "single_thread": {"value": v1, "cores": 1,
                              "sample": f"the first {n_single} instances, one iteration each "
                                        f"({sum(w.K * w.T for w in one):.3g} rollout-steps, "
                                        f"{t1:.1f} s)"},
            **info}


def cpu_baseline_single(wl, iters: int) -> dict:
    """One thread on the whole workload (iters iterations), and the rollouts
    of one iteration split over the host threads by sample range."""
    from oracle import oracle as O
    t0 = time.perf_counter()
    O.mppi(wl, iters=iters)
    t1 = time.perf_counter() - t0
    eps = O.workload_noise(wl)
    thr = O.host_threads()
    t0 = time.perf_counter()
    S = O.rollout_costs_parallel(wl, eps, threads=thr)
    O.softmin_update(wl, S, eps)
    tn = time.perf_counter() - t0
    info = host_info()
    return {"value": wl.K * wl.T / tn, "unit": "rollout-steps/s", "cores": thr, "kind": "oracle",
            "sample": f"{wl.name}: K {wl.K}, T {wl.T}, one iteration, the rollouts split over "
                      f"{thr} threads by sample range (binary64 C oracle, {tn:.2f} s)",
            "single_thread": {"value": iters * wl.K * wl.T / t1, "cores": 1,
                              "sample": f"{iters} iterations, one thread ({t1:.1f} s)"},
            **info}


# ---------------------------------------------------------------------------
# GPU workloads
# ---------------------------------------------------------------------------
def run_single(args, wl, update_forms: bool = False, autotune_reps: int = 30) -> dict:
    """One context, `wl.iters` warm-started iterations per step."""
    import torch
    import paper_2409_07563_amd as M
    I = wl.iters
    ctl = M.Controller(wl, device="cuda:0")
    stream = ctl.stream
    tuned = None
    if args.tuning:
        ctl.set_tuning(**json.loads(args.tuning))
    elif not args.no_autotune:
        tuned = ctl.autotune(reps=autotune_reps)
    # each step calls the C ABI directly on the library's stream (ordered once
    # after torch's stream here, not re-synchronised with it in every step)
    L = M.lib()
    ctl._enter()

    def step():
        M._abi.check(L.mppi_iterate(ctl.ctx, I))
    s = timed(stream, step, args.steps, args.warmup)
    steps_per_iter = wl.K * wl.T
    out = {"workload": wl.name, "K": wl.K, "T": wl.T, "iterations_per_step": I,
           "dynamics": wl.model, "integrator": wl.integrator, "cost": wl.cost,
           "value": I * steps_per_iter / s, "ms_per_step": s * 1e3,
           "us_per_iteration": s * 1e6 / I}
    if wl.cx is not None:
        out["obstacles"] = len(wl.cx)
    chosen = ctl.tuning()
    if update_forms:
        # the per-phase form with each update form, and the iteration forms
        forms = {}
        for form, name in ((0, "two_pass"), (1, "one_pass"), (2, "chunked")):
            try:
                ctl.set_tuning(update_form=form, batch_form=0)
            except M.MPPIError:
                continue
            forms[name] = timed(stream, step, args.steps, max(1, args.warmup)) * 1e3
        ctl.set_tuning(**chosen)
        out["update_forms_ms_per_step"] = forms
        iforms = {}
        for bf, name in ((0, "phases"), (1, "one_launch")):
            try:
                ctl.set_tuning(batch_form=bf)
            except M.MPPIError:
                continue
            iforms[name] = timed(stream, step, args.steps, max(1, args.warmup)) * 1e3
        ctl.set_tuning(**chosen)
        if len(iforms) > 1:
            out["iteration_forms_ms_per_step"] = iforms
    t_noise, t_roll, t_upd = phase_times(ctl, args.kernel_reps)
    ops_step = rollout_ops_per_step(wl)
    tune = ctl.tuning()
    fused = tune["batch_form"] == 1
    if fused:
        # the whole iteration is one launch: its duration from ten iterations
        # replayed from one graph (an upper bound: the gaps between launches
        # are counted)
        t_roll = timed(stream, lambda: ctl.iterate(10), max(1, args.steps // 5),
                       max(1, args.warmup // 5)) / 10
    achieved = ops_step * steps_per_iter / t_roll
    split = tune["rollout_form"] == 1
    scan = tune["rollout_form"] == 2
    lanes = tune["lanes_per_sample"]
    kernel = ("di_iteration_kernel (the whole iteration)" if fused else
              "split_dynamics + split_cost" if split else
              "rollout_bicycle_scan_kernel" if scan else
              "rollout_bicycle_group_kernel" if lanes > 1 else "rollout_kernel")
    traffic = traffic_record("rollout", args.workload if args.workload != "all" else
                             {"c3_quadrotor": "c3", "c2_bicycle_circles": "c2_circles"}.get(
                                 wl.name, wl.name),
                             "scan_kernel<" if scan else
                             f", {lanes}>" if lanes > 1 else "rollout_kernel<")
    out["roofline"] = {
        "bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
        "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS,
        "traffic": None if (split or fused) else traffic,
        "kernel": kernel,
        "ops_per_rollout_step": ops_step, "launch_us": t_roll * 1e6}
    eps_bytes = 4 * wl.T * wl.m * wl.K
    out["kernels"] = {
        "noise": {"us": t_noise * 1e6, "hbm_GBps": eps_bytes / t_noise / 1e9},
        "rollout": {"us": t_roll * 1e6},
        "softmin_update": {"us": t_upd * 1e6, "hbm_GBps": (eps_bytes + 8 * wl.K) / t_upd / 1e9}}
    out["tuning"] = tune
    if tuned:
        out["rollout_forms_us"] = rollout_forms(tuned)
    ctl.close()
    return out


def run_grad(args, wl, full: bool = True) -> dict:
    """Differentiable MPPI (MLP residual dynamics): the plain forward
    iteration, and one forward iteration in gradient mode (checkpointing
    rollout) plus the adjoint backward of L = |U - u_ref|^2, on the same GPU."""
    import torch
    import paper_2409_07563_amd as M
    import workloads as W

    dev = torch.device("cuda:0")
    uref = torch.as_tensor(W.c5_uref(T=wl.T), device=dev)
    L = M.lib()

    u_start = torch.as_tensor(wl.u0, device=dev).contiguous()

    def configured(c):
        # every timed step is the configured iteration: iteration word 0
        # from the nominal controls u0 (so the samples of nonzero weight,
        # which the backward sweeps, are the same in every step)
        M._abi.check(L.mppi_set_controls(c.ctx, u_start.data_ptr()))
        M._abi.check(L.mppi_set_iteration(c.ctx, 0))
        M._abi.check(L.mppi_iterate(c.ctx, 1))

    def measure(w, three: bool):
        plain = M.Controller(w, device=dev)
        if not args.no_autotune:
            plain.autotune(reps=10)
        tuning = plain.tuning()
        plain._enter()
        t_fwd = timed(plain.stream, lambda: configured(plain), args.steps, args.warmup)
        t_noise, t_roll, t_upd = phase_times(plain, args.kernel_reps)
        plain.close()
        grad = M.Controller(w, device=dev, requires_grad=True)
        # the same launch shapes as the plain forward (the gradient mode has
        # the two-pass update only: its adjoint reads the stored weights)
        grad.set_tuning(**{k: v for k, v in tuning.items() if k != "update_form"})
        grad._enter()
        configured(grad)
        G = (2.0 * (grad.controls() - uref)).contiguous()
        out = torch.empty(grad.theta_len(), device=dev)

        def fwd_bwd():
            configured(grad)
            M._abi.check(L.mppi_backward(grad.ctx, G.data_ptr(), out.data_ptr()))
        t_fb = timed(grad.stream, fwd_bwd, args.steps, args.warmup)
        t_fg = timed(grad.stream, lambda: configured(grad), args.steps, args.warmup)
        swept = int((grad.weights() > 0).sum())
        res = dict(t_fwd=t_fwd, t_noise=t_noise, t_roll=t_roll, t_upd=t_upd, t_fb=t_fb,
                   t_fg=t_fg, swept=swept, tuning=tuning)
        if three:
            # the same backward with the per-tile sweep over the whole horizon
            # (the segment-parallel mode switched off), for comparison
            grad.set_tuning(adjoint_tiles=0)
            grad._enter()
            res["t_fb_tile"] = timed(grad.stream, fwd_bwd, args.steps, args.warmup)
            grad.set_tuning(adjoint_tiles=tuning["adjoint_tiles"])
            grad._enter()
        if three:
            # three warm-started iterations and the reverse pass through all
            # of them (rebuilds each iteration from the tape, then its adjoint)
            du0 = torch.empty(w.T * w.m, device=dev)
            u0 = torch.as_tensor(w.u0, device=dev).contiguous()

            def fwd3():
                M._abi.check(L.mppi_set_controls(grad.ctx, u0.data_ptr()))
                M._abi.check(L.mppi_iterate(grad.ctx, 3))

            def fwd3_bwd():
                fwd3()
                M._abi.check(L.mppi_backward_iters(grad.ctx, G.data_ptr(), out.data_ptr(),
                                                   du0.data_ptr()))
            res["t_f3"] = timed(grad.stream, fwd3, args.steps, args.warmup)
            res["t_f3b"] = timed(grad.stream, fwd3_bwd, args.steps, args.warmup)
        grad.close()
        return res

    r = measure(wl, full)
    steps = wl.K * wl.T
    flops = 2.0 * mlp_macs(wl.mlp_hidden) * steps
    achieved = flops / r["t_roll"]
    eps_bytes = 4 * wl.T * wl.m * wl.K
    out = {"workload": wl.name, "K": wl.K, "T": wl.T, "iterations_per_step": 1,
           "dynamics": wl.model, "hidden": wl.mlp_hidden, "integrator": wl.integrator,
           "cost": wl.cost, "lambda": wl.lam, "checkpoint_every": 10,
           "value": steps / r["t_fwd"], "ms_per_step": r["t_fwd"] * 1e3,
           "fwd_bwd_over_fwd": r["t_fb"] / r["t_fwd"],
           "grad": {"fwd_plain_ms": r["t_fwd"] * 1e3, "fwd_checkpointing_ms": r["t_fg"] * 1e3,
                    "fwd_plus_bwd_ms": r["t_fb"] * 1e3, "bwd_ms": (r["t_fb"] - r["t_fg"]) * 1e3,
                    "samples_swept": r["swept"]},
           "roofline": {"bound": "mfma", "achieved": achieved / 1e12,
                        "peak": MFMA_FP32_PEAK / 1e12, "unit": "TFLOP/s",
                        "frac": achieved / MFMA_FP32_PEAK,
                        "traffic": traffic_record("rollout_tile", "c5"),
                        "kernel": "rollout_tile_kernel",
                        "flops_per_rollout_step": 2 * mlp_macs(wl.mlp_hidden),
                        "launch_us": r["t_roll"] * 1e6},
           "kernels": {"noise": {"us": r["t_noise"] * 1e6,
                                 "hbm_GBps": eps_bytes / r["t_noise"] / 1e9},
                       "rollout": {"us": r["t_roll"] * 1e6},
                       "softmin_update": {"us": r["t_upd"] * 1e6,
                                          "hbm_GBps": (eps_bytes + 8 * wl.K) / r["t_upd"] / 1e9}},
           "tuning": r["tuning"]}
    if full:
        out["grad"]["bwd_forms_ms"] = {"segment_parallel": (r["t_fb"] - r["t_fg"]) * 1e3,
                                       "per_tile": (r["t_fb_tile"] - r["t_fg"]) * 1e3}
        out["grad"]["fwd_bwd_over_fwd_per_tile"] = r["t_fb_tile"] / r["t_fwd"]
        out["grad"]["three_iterations"] = {"fwd_ms": r["t_f3"] * 1e3,
                                           "fwd_plus_bwd_ms": r["t_f3b"] * 1e3,
                                           "fwd_bwd_over_fwd": r["t_f3b"] / r["t_f3"]}
        d = measure(wl.replace(lam=500.0), False)
        out["grad"]["lambda_500"] = {"fwd_bwd_over_fwd": d["t_fb"] / d["t_fwd"],
                                     "fwd_plus_bwd_ms": d["t_fb"] * 1e3,
                                     "bwd_ms": (d["t_fb"] - d["t_fg"]) * 1e3,
                                     "samples_swept": d["swept"]}
    # the bfloat16 mode of the MLP (bfloat16 operands, binary32 accumulation)
    b = measure(wl.replace(mlp_bf16=1), False)
    out["bf16"] = {"ms_per_step": b["t_fwd"] * 1e3, "value": steps / b["t_fwd"],
                   "fwd_bwd_over_fwd": b["t_fb"] / b["t_fwd"],
                   "fwd_plus_bwd_ms": b["t_fb"] * 1e3, "bwd_ms": (b["t_fb"] - b["t_fg"]) * 1e3,
                   "rollout_us": b["t_roll"] * 1e6,
                   "rollout_speedup_over_fp32": r["t_roll"] / b["t_roll"],
                   "mfma_TFLOPs": flops / b["t_roll"] / 1e12,
                   "frac_of_bf16_peak": flops / b["t_roll"] / MFMA_BF16_PEAK,
                   "tuning": b["tuning"]}
    return out


def run_batch(args, insts, loop_baseline: bool = True) -> dict:
    """Many independent instances: one batched context (one launch per phase,
    the per-iteration sequence replayed from a hipGraph) against the same
    instances run one context after another on one stream."""
    import paper_2409_07563_amd as M
    total = sum(w.K * w.T for w in insts)
    ctl = M.Controller(insts, device="cuda:0")
    stream = ctl.stream
    if args.tuning:
        ctl.set_tuning(**json.loads(args.tuning))
    elif not args.no_autotune:
        ctl.autotune(reps=3)
    tuning = ctl.tuning()
    L = M.lib()
    ctl._enter()

    def step():  # the C ABI directly on the library's stream
        M._abi.check(L.mppi_iterate(ctl.ctx, 1))
    # both batch forms timed on their own (one warm-started iteration per
    # step): four launches per iteration, and the one-launch form
    forms = {}
    for form, name, extra in ((0, "phases", {}),
                              (1, "one_launch", {"batch_tile": 256, "update_form": 0})):
        try:
            ctl.set_tuning(batch_form=form, **extra)
        except M.MPPIError:
            continue
        forms[name] = timed(stream, step, max(1, args.steps // 2),
                            max(1, args.warmup // 2)) * 1e3
    ctl.set_tuning(**tuning)
    s = timed(stream, step, args.steps, args.warmup)
    tn, tr, tu = phase_times(ctl, max(1, args.kernel_reps // 5))
    ctl.close()
    out = {"workload": "c4_batched_bicycle", "instances": len(insts), "sum_K_T": total,
           "K_range": [min(w.K for w in insts), max(w.K for w in insts)],
           "T_range": [min(w.T for w in insts), max(w.T for w in insts)],
           "obstacles_range": [min(len(w.cx) for w in insts), max(len(w.cx) for w in insts)],
           "iterations_per_step": 1, "dynamics": insts[0].model, "cost": insts[0].cost,
           "value": total / s, "ms_per_step": s * 1e3, "tuning": tuning,
           "batch_forms_ms_per_step": forms}
    if loop_baseline:
        # the same instances as single contexts, one after another on one
        # stream (each with the default launch shapes of its size)
        singles = [M.Controller(w, device="cuda:0", stream=stream) for w in insts]
        singles[0]._enter()

        def loop():
            for c in singles:
                M._abi.check(L.mppi_iterate(c.ctx, 1))
        s_loop = timed(stream, loop, max(1, args.steps // 4), 1)
        for c in singles:
            c.close()
        out["looped_single_contexts"] = {"ms_per_step": s_loop * 1e3, "value": total / s_loop,
                                         "speedup_of_batch": s_loop / s}
    ops = sum(rollout_ops_per_step(w) * w.K * w.T for w in insts)
    achieved = ops / tr
    eps_bytes = sum(4 * w.T * w.m * w.K for w in insts)
    out["roofline"] = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                       "unit": "Tops/s", "frac": achieved / VALU_PEAK_OPS,
                       "traffic": traffic_record("rollout", "c4"),
                       "kernel": "batch_rollout_kernel",
                       "ops_per_rollout_step": rollout_ops_per_step(insts[0]),
                       "launch_us": tr * 1e6}
    out["kernels"] = {"noise": {"us": tn * 1e6, "hbm_GBps": eps_bytes / tn / 1e9},
                      "rollout": {"us": tr * 1e6},
                      "softmin_update": {"us": tu * 1e6, "hbm_GBps": eps_bytes / tu / 1e9}}
    return out


def headline_line(args, lead: dict, **extra) -> dict:
    out = {"metric": METRIC, "value": lead["value"], "unit": "rollout-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": lead["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic"}
    out.update(extra)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="all",
                    help="all (default: the batched headline with every leg), or one of "
                         "c1, c2_circles, c2_costmap, c3, c4, c5 on its own")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--cpu-iters", type=int, default=None,
                    help="oracle iterations for a single workload's CPU baseline")
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
        print("bench.py measures one GPU: this build runs on a single GPU and has no "
              "multi-GPU path (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
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

    if args.workload == "all":
        return main_all(args)

    wl = make_workload(args.workload)
    if args.cost_cosines:
        wl = ([w.replace(cost_cosines=args.cost_cosines) for w in wl] if isinstance(wl, list)
              else wl.replace(cost_cosines=args.cost_cosines))
    if isinstance(wl, list):
        r = run_batch(args, wl)
        line = headline_line(args, r, config={k: r[k] for k in (
            "workload", "instances", "sum_K_T", "K_range", "T_range", "obstacles_range",
            "iterations_per_step", "cost")}, **{k: v for k, v in r.items() if k in (
                "tuning", "looped_single_contexts", "roofline", "kernels",
                "batch_forms_ms_per_step")})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_batch(wl, 8, 128)
    elif wl.model == "bicycle_mlp":
        r = run_grad(args, wl)
        line = headline_line(args, r, config={k: r[k] for k in (
            "workload", "K", "T", "iterations_per_step", "dynamics", "hidden", "integrator",
            "cost", "lambda", "checkpoint_every")}, **{k: r[k] for k in (
                "fwd_bwd_over_fwd", "grad", "roofline", "kernels", "tuning", "bf16")})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_single(wl, 1)
    else:
        r = run_single(args, wl, update_forms=True)
        line = headline_line(args, r, config={k: r[k] for k in (
            "workload", "K", "T", "iterations_per_step", "dynamics", "integrator", "cost")
            if k in r}, **{k: v for k, v in r.items() if k in (
                "roofline", "kernels", "tuning", "rollout_forms_us", "update_forms_ms_per_step",
                "iteration_forms_ms_per_step")})
        line["config"]["cost_cosines"] = int(getattr(wl, "cost_cosines", 0))
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline_single(wl, args.cpu_iters or wl.iters)
        line["achievable"] = {"hbm_copy_GBps": copy_bandwidth()}
    print(json.dumps(line), flush=True)


def main_all(args):
    """The headline (the batched instances) and every leg, one JSON line."""
    import workloads as W
    t_all = time.perf_counter()
    ceil = measure_ceilings()
    print("[bench] ceilings measured", file=sys.stderr, flush=True)
    insts = W.c4()
    lead = run_batch(args, insts)
    print(f"[bench] c4 batch: {lead['value']:.4g} rollout-steps/s", file=sys.stderr, flush=True)
    c3 = run_single(args, W.c3(), autotune_reps=10)
    print(f"[bench] c3: {c3['value']:.4g}", file=sys.stderr, flush=True)
    c2 = run_single(args, W.c2("circles"), autotune_reps=30)
    print(f"[bench] c2: {c2['value']:.4g}", file=sys.stderr, flush=True)
    c5 = run_grad(args, W.c5(), full=False)
    print(f"[bench] c5: fwd+bwd/fwd {c5['fwd_bwd_over_fwd']:.3f}", file=sys.stderr, flush=True)
    c1 = run_single(args, W.c1(), autotune_reps=30)
    # latency references: one iteration's steps as a dependent chain on one
    # wave, and an empty three-kernel graph launch (steps here are direct
    # launches, pipelined on the stream, so a launch's own latency overlaps
    # the previous iteration)
    c1["floors_us"] = {"chain_T100": ceil["chain_us"]["T100"],
                       "empty_3_kernel_graph": ceil["graph_launch_us"]["3_kernels"]}
    c1["us_per_iteration_over_chain"] = c1["us_per_iteration"] / ceil["chain_us"]["T100"]
    print(f"[bench] c1: {c1['value']:.4g}", file=sys.stderr, flush=True)
    cfg = {k: lead[k] for k in ("workload", "instances", "sum_K_T", "K_range", "T_range",
                                "obstacles_range", "iterations_per_step", "dynamics", "cost")}
    cfg["legs"] = ["c3_quadrotor", "c2_bicycle_circles", "c5_bicycle_mlp", "c1_double_integrator"]
    line = headline_line(args, lead, config=cfg,
                         fwd_bwd_over_fwd=c5["fwd_bwd_over_fwd"],
                         roofline=lead["roofline"], kernels=lead["kernels"],
                         tuning=lead["tuning"],
                         looped_single_contexts=lead.get("looped_single_contexts"),
                         batch_forms_ms_per_step=lead.get("batch_forms_ms_per_step"),
                         legs={"c3": c3, "c2": c2, "c5": c5, "c1": c1},
                         ceilings=ceil)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(insts, 8, 128)
    line["wall_s"] = time.perf_counter() - t_all
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

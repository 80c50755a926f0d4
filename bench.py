"""Benchmark of the FP64 finite-volume Euler step on one MI355X.

Workload: 2D Euler, 2048 x 2048 periodic grid on [0,10]^2, isentropic vortex
(beta 5, Mach 0.5 diagonal) plus 32 seeded Gaussian density bumps (amplitude
1e-2), MUSCL-minmod + Roe, SSP-RK3, CFL 0.5. One "step" is one full SSP-RK3
time step (3 stages + the CFL reduction) through ``fv_step``.

Sequence:
  1. K timed steps with the default launch table;
  2. the autotuner (the paper's method): ~300 sampled launch vectors timed,
     network trained on 75 %, whole space predicted on the GPU, top 8
     re-measured; default / tuned / best-of-random compared interleaved;
  3. K timed steps with the tuned launch table -> `value`;
  4. per-kernel durations of the tuned step from HIP events the library
     records around each launch on its own stream -> `roofline`;
  5. adjoint vs primal cost on the 512^2 / 60-step adjoint workload;
  6. the FP64 CPU oracle on the host cores for a bounded sample.
Prints ONE JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--samples N] [--no-cpu] [--no-tune]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

HBM_PEAK_GBPS = 8000.0
METRIC = "cell-updates/s + HBM GB/s vs peak, tuned vs default launch; adjoint/primal"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048, help="cells per side")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--samples", type=int, default=300, help="timed launch vectors for the tuner")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-fused", action="store_true", help="skip the fused single-grid and batch measurements")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--launch", type=str, default=None, help="14 launch parameters as a JSON list (skips tuning)")
    ap.add_argument("--timing-steps", type=int, default=20)
    return ap.parse_args()


def timed_steps(torch, solver, U0, launch, steps, warmup):
    """ms per step over `steps` steps from U0 (inputs resident in HBM)."""
    solver.set_launch(launch)
    solver.set_state(U0)
    solver.step(warmup)
    solver.set_state(U0)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    rc, flags = solver.status()
    if flags:
        log(f"non-physical flags {flags}")
        sys.exit(3)
    return e0.elapsed_time(e1) / steps


def kernel_table(solver, g, launch, steps, fv, traffic):
    solver.set_launch(launch)
    solver.set_timing(True)
    solver.step(steps)
    ms, cnt = solver.get_timing()
    solver.set_timing(False)
    sb = traffic.site_bytes(g)
    total = sum(ms)
    kernels = {}
    for i, name in enumerate(fv.SITES):
        if cnt[i] == 0:
            continue
        avg_ms = ms[i] / cnt[i]
        kernels[name] = {
            "avg_us": round(avg_ms * 1e3, 3),
            "launches_per_step": cnt[i] / steps,
            "share": round(ms[i] / total, 4),
            "alg_bytes": sb[name],
            "achieved_GBps": round(sb[name] / (avg_ms * 1e-3) / 1e9, 1),
        }
    return kernels


def adjoint_ratio(torch, fv, inputs):
    """fv_adjoint_step / fv_step per step, and the checkpointed reverse / forward,
    on the 512^2 vortex, 60 steps, checkpoints every 10."""
    from paper_2306_14011_amd.rollout import pressure_integral, rollout
    g, U0 = inputs.vortex_case(512, seed=0)
    s = fv.Solver(g)
    s.set_state(U0)
    dts = torch.zeros(60, dtype=torch.float64, device="cuda")
    s.step(60, dt_out=dts)
    torch.cuda.synchronize()
    lam = torch.ones(g.shape, dtype=torch.float64, device="cuda")
    Ustate = s.U.clone()
    stream = torch.cuda.current_stream()

    def timeit(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    s.U.copy_(Ustate)
    t_primal = timeit(lambda: s.step(1, dt_in=dts[:1]), 50)
    t_adj = timeit(lambda: fv.fv_adjoint_step(s.ctx, Ustate.data_ptr(), dts[:1].data_ptr(), lam.data_ptr()), 50)
    x = torch.as_tensor(U0).cuda()
    window = inputs.adjoint_window(512, 64)

    def fwd():
        with torch.no_grad():
            rollout(x, s, 60, every=10)

    def fwd_bwd():
        xr = x.clone().requires_grad_(True)
        out, _ = rollout(xr, s, 60, every=10)
        pressure_integral(out, g, window).backward()

    t_fwd = timeit(fwd, 3)
    t_fb = timeit(fwd_bwd, 3)
    s.close()
    return {
        "workload": "512x512 vortex, 60 steps, checkpoints every 10, J = pressure over cells [224,288)^2",
        "primal_step_ms": round(t_primal, 4),
        "adjoint_step_ms": round(t_adj, 4),
        "adjoint_over_primal_step": round(t_adj / t_primal, 3),
        "forward_60_ms": round(t_fwd, 3),
        "reverse_60_ms_incl_recompute": round(t_fb - t_fwd, 3),
        "reverse_over_forward": round((t_fb - t_fwd) / t_fwd, 3),
    }


def fused_single(torch, fv, traffic, g, U0, steps, warmup):
    """The fused path on the same grid: segment heights swept, best kept."""
    s = fv.Solver(g)
    res = {}
    for seg in (8, 16, 32, 64):
        s.set_path(fv.FV_PATH_FUSED, seg, 0)
        res[seg] = timed_steps(torch, s, U0, fv.fv_default_launch(), steps, warmup)
    seg = min(res, key=res.get)
    s.set_path(fv.FV_PATH_FUSED, seg, 0)
    s.set_timing(True)
    s.step(20)
    ms, cnt = s.get_timing()
    s.set_timing(False)
    s.close()
    avg_ms = ms[7] / cnt[7]
    alg = traffic.fused_step_bytes(g) / 3.0   # per stage launch, averaged over the three
    return {
        "ms_per_step": res[seg],
        "value": g.ncells / (res[seg] * 1e-3),
        "seg": seg,
        "ms_per_step_by_seg": {str(k): round(v, 4) for k, v in res.items()},
        "stage_avg_us": round(avg_ms * 1e3, 2),
        "stage_alg_bytes": alg,
        "stage_achieved_GBps": round(alg / (avg_ms * 1e-3) / 1e9, 1),
        "alg_bytes_per_cell_update": traffic.fused_step_bytes(g) / g.ncells,
    }


def batch_bench(torch, fv, inputs, steps):
    """96 uneven periodic vortex grids (sides 128..1024), fused stages in a HIP graph."""
    spec = inputs.batch_case(count=96, seed=0)
    cells = sum(gg.ncells for gg in spec.grids)
    best = None
    for seg, order in ((16, 1), (32, 1), (16, 0)):
        B = fv.Batch(spec.grids, seg=seg, order=order)
        B.set_states(spec.states)
        B.step(3)
        torch.cuda.synchronize()
        B.set_states(spec.states)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        stream = torch.cuda.current_stream()
        e0.record(stream)
        B.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        rc, flags = B.status()
        if flags:
            log(f"batch flags {flags}")
        if best is None or ms < best[0]:
            best = (ms, seg, order, B)
        else:
            B.close()
    ms, seg, order, B = best
    # device-clock record of 20 steps: per-grid step time = sum over stages of (last end - first start)
    B.set_states(spec.states)
    tpu = B.set_timing(20)
    B.step(20)
    torch.cuda.synchronize()
    clk = B.clocks()
    B.close()
    per = (clk[..., 1] - clk[..., 0]).sum(axis=2) / tpu   # (steps, grids) microseconds
    import numpy as np
    # sequential baseline: each grid alone through the single-grid fused path
    seq = 0.0
    for gg, st in zip(spec.grids, spec.states):
        s = fv.Solver(gg)
        s.set_path(fv.FV_PATH_FUSED, 16, 0)
        seq += timed_steps(torch, s, st, fv.fv_default_launch(), 5, 1)
        s.close()
    return {
        "workload": "96 periodic 2D vortex grids, sides U{128..1024}, beta U[1,5], FP64, 3 fused stages per step in a HIP graph",
        "cells": cells,
        "ms_per_step": round(ms, 4),
        "value": cells / (ms * 1e-3),
        "unit": "cell-updates/s",
        "seg": seg,
        "order": "largest_first" if order == 1 else "given",
        "per_grid_step_us_p50": round(float(np.percentile(per, 50)), 2),
        "per_grid_step_us_p99": round(float(np.percentile(per, 99)), 2),
        "sequential_single_grid_ms_per_step": round(seq, 4),
        "batch_speedup_vs_sequential": round(seq / ms, 3),
    }


def cpu_baseline(g, U0, seconds):
    """The oracle as it stands, on the host cores, for about `seconds`."""
    import oracle
    steps = 0
    U = U0
    t0 = time.perf_counter()
    while True:
        U, _, _ = oracle.run(g, U, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return {
        "value": g.ncells * steps / el,
        "unit": "cell-updates/s",
        "cores": oracle.omp_threads(),
        "kind": "oracle",
        "sample": f"{steps} SSP-RK3 steps of the {g.n[0]}x{g.n[1]} workload (FP64, OpenMP over cells), {el:.1f} s",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2306_14011_amd import fv, inputs, traffic

    g, U0 = inputs.vortex_bumps_case(a.n, seed=a.seed)
    log(f"workload {a.n}x{a.n} vortex+bumps, steps {a.steps}, warmup {a.warmup}")
    default = fv.fv_default_launch()
    s = fv.Solver(g)
    ms_default = timed_steps(torch, s, U0, default, a.steps, a.warmup)
    log(f"default launch: {ms_default:.4f} ms/step")

    tune = None
    launch = default
    if a.launch:
        launch = json.loads(a.launch)
    elif not a.no_tune:
        from paper_2306_14011_amd.autotune import Autotuner
        t0 = time.perf_counter()
        at = Autotuner(g, U0, seed=a.seed, repeats=3, warmup=3, min_ms=20.0)
        tune = at.run(count=a.samples, k=8, rounds=5)
        at.close()
        tune["tuning_seconds"] = round(time.perf_counter() - t0, 1)
        launch = tune["tuned_launch"]
        log(f"tuned in {tune['tuning_seconds']} s: R2(test) {tune['r2_test']:.3f}, "
            f"default/tuned {tune['factor_vs_default']:.3f}, best-random/tuned {tune['factor_vs_best_random']:.3f}")

    ms_tuned = timed_steps(torch, s, U0, launch, a.steps, a.warmup)
    value = g.ncells / (ms_tuned * 1e-3)
    log(f"tuned launch {launch}: {ms_tuned:.4f} ms/step")

    kernels = kernel_table(s, g, launch, a.timing_steps, fv, traffic)
    dom = max(kernels, key=lambda k: kernels[k]["share"])
    ach = kernels[dom]["achieved_GBps"]
    roofline = {
        "bound": "hbm",
        "achieved": ach,
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBPS, 4),
        "traffic": None,
        "kernel": dom,
    }
    step_b = traffic.step_bytes(g)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_tuned,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D Euler {a.n}x{a.n} periodic vortex + 32 Gaussian bumps, MUSCL-minmod/Roe/SSP-RK3, CFL 0.5",
            "cells": g.ncells,
            "path": "split 7-kernel step, MLP-tuned launch" if tune else "split 7-kernel step",
            "launch": launch,
        },
        "roofline": roofline,
        "default_launch": {"launch": default, "ms_per_step": ms_default,
                           "value": g.ncells / (ms_default * 1e-3)},
        "tuned_over_default": round(ms_default / ms_tuned, 4),
        "step_effective_GBps": round(step_b * value / g.ncells / 1e9, 1),
        "alg_bytes_per_cell_update": step_b / g.ncells,
        "kernels": kernels,
    }
    if tune:
        out["autotune"] = {k: v for k, v in tune.items() if k not in ("top_pred",)}
    s.close()
    if not a.no_fused:
        out["fused"] = fused_single(torch, fv, traffic, g, U0, a.steps, a.warmup)
        log(f"fused path: {out['fused']['ms_per_step']:.4f} ms/step (seg {out['fused']['seg']})")
        out["batch"] = batch_bench(torch, fv, inputs, 100)
        log(f"batch: {out['batch']['value']:.3e} cell-updates/s")
    if not a.no_adjoint:
        out["adjoint"] = adjoint_ratio(torch, fv, inputs)
        log(f"adjoint/primal per step {out['adjoint']['adjoint_over_primal_step']}")
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, U0, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the FP64 finite-volume Euler step on one MI355X.

Workload: 2D Euler, 2048 x 2048 periodic grid on [0,10]^2, isentropic vortex
(beta 5, Mach 0.5 diagonal) plus 32 seeded Gaussian density bumps (amplitude
1e-2), MUSCL-minmod + Roe, SSP-RK3, CFL 0.5. One "step" is one full SSP-RK3
time step (3 stages + the CFL reduction) through ``fv_step``.

Prints ONE JSON line: cell-updates/s over K timed steps (inputs resident in
HBM), the dominant kernel's achieved bandwidth against the 8 TB/s HBM peak
(per-kernel durations from HIP events recorded by the library on its own
stream), and the FP64 CPU oracle timed on the host on a bounded sample.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--launch JSON]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HBM_PEAK_GBPS = 8000.0
METRIC = "cell-updates/s + HBM GB/s vs peak, tuned vs default launch; adjoint/primal"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=2048, help="cells per side")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--launch", type=str, default=None, help="14 launch parameters as a JSON list")
    ap.add_argument("--timing-steps", type=int, default=20)
    return ap.parse_args()


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
        "sample": f"{steps} SSP-RK3 steps of the {g.n[0]}x{g.n[1]} workload (FP64, OpenMP), {el:.1f} s",
    }


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2306_14011_amd import fv, inputs, traffic

    g, U0 = inputs.vortex_bumps_case(a.n, seed=a.seed)
    print(f"[bench] workload {a.n}x{a.n} vortex+bumps, steps {a.steps}, warmup {a.warmup}", file=sys.stderr,
          flush=True)
    s = fv.Solver(g)
    if a.launch:
        s.set_launch(json.loads(a.launch))
    launch = s.get_launch()
    s.set_state(U0)
    dev = torch.device("cuda")
    stream = torch.cuda.current_stream(dev)

    s.step(a.warmup)
    torch.cuda.synchronize()
    s.set_state(U0)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    s.step(a.steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    rc, flags = s.status()
    if flags:
        print(f"[bench] non-physical flags {flags}", file=sys.stderr)
        sys.exit(3)
    ms_per_step = gpu_ms / a.steps
    value = g.ncells * a.steps / (gpu_ms * 1e-3)
    print(f"[bench] timed {a.steps} steps: {gpu_ms:.1f} ms (wall {wall * 1e3:.1f} ms)", file=sys.stderr, flush=True)

    # per-kernel durations: HIP events recorded by the library around each launch
    s.set_timing(True)
    s.step(a.timing_steps)
    ms, cnt = s.get_timing()
    s.set_timing(False)
    sb = traffic.site_bytes(g)
    kernels = {}
    for i, name in enumerate(fv.SITES):
        if cnt[i] == 0:
            continue
        avg_ms = ms[i] / cnt[i]
        kernels[name] = {
            "avg_us": round(avg_ms * 1e3, 3),
            "launches_per_step": cnt[i] / a.timing_steps,
            "share": ms[i] / sum(ms),
            "alg_bytes": sb[name],
            "achieved_GBps": round(sb[name] / (avg_ms * 1e-3) / 1e9, 1),
        }
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
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D Euler {a.n}x{a.n} periodic vortex+32 Gaussian bumps, MUSCL-minmod/Roe/SSP-RK3, CFL 0.5",
            "cells": g.ncells,
            "path": "split 7-kernel step",
            "launch": launch,
        },
        "roofline": roofline,
        "step_effective_GBps": round(step_b * value / g.ncells / 1e9, 1),
        "alg_bytes_per_cell_update": step_b / g.ncells,
        "kernels": kernels,
    }
    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, U0, a.cpu_seconds)
    s.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

#!/usr/bin/env python3
"""Benchmark: MHD cell-updates/s of the fused HIP path on a 256^3 periodic box.

Workload (synthetic, seeded): 256^3 periodic unit cube, gamma = 5/3, rho = 1,
p = 0.6, uniform B = (0.2, 0, 0), solenoidal Gaussian velocity with a shell
spectrum peaked at k = 4 and rms Mach 0.5; HLLD + PLM (van Leer) + E^c CT + RK2,
CFL 0.3.  A step is one full RK2 cycle (two fused stage launches and the
device-side cycle control) over the whole box; a cell-update is one cell
advanced one cycle.  Inputs are resident in HBM before timing starts.

The line reports FP64 as ``value`` (the paper's precision) and the FP32 run
under ``fp32``; each carries its own roofline for the stage kernel:
algorithmic HBM bytes per cell and cycle are 40 state words (stage 1 reads 8
and writes 8; stage 2 reads 8 + 8 and writes 8), i.e. 320 B (FP64) and 160 B
(FP32), against the 8 TB/s HBM3E peak of the MI355X.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 256
METRIC = "MHD cell-updates/s at 256^3 (FP64 vs FP32, %HBM peak); batched p50/p99 latency"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mhd_device.h", "mhd_stage.inl", "mhd_stage_launch.inl", "mhd_internal.h"):
        with open(os.path.join(ROOT, "paper_2304_13746_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(precision: str):
    """HBM bytes per stage launch from the committed rocprofv3 counter summary,
    or None if the summary is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"stage_kernel_256_{precision}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel source hash: ([0-9a-f]+)", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"HBM bytes per stage launch \(scaled\): ([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def run_gpu(state, precision: str, steps: int, warmup: int, tile: int = 0, zchunk: int = 0):
    import torch

    from paper_2304_13746_amd.box import MHDBox

    box = MHDBox(N, N, N, precision=precision, riemann="hlld", tile=tile, zchunk=zchunk)
    box.set_state(state)
    box.step(warmup)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(box.stream)
    box.step(steps)
    stop.record(box.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    _, t, dt, rc = box.get_state(check=False)
    box.close()
    return {"ms_total": ms, "wall_s": wall, "t": t, "dt_next": dt, "rc": rc}


def roofline(precision: str, ms_per_step: float):
    word = 8 if precision == "fp64" else 4
    cells = N ** 3
    # two stage launches per cycle: 16 and 24 state words per cell -> 20 on average
    bytes_per_launch = 20 * word * cells
    launch_s = ms_per_step * 1e-3 / 2.0
    achieved = bytes_per_launch / launch_s / 1e9
    traffic = counter_traffic(precision)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 4),
            "traffic_unit": "GB per stage launch",
            "algorithmic_bytes_per_launch": bytes_per_launch}


def cpu_baseline(state):
    """The FP64 oracle on the host cores: 2 RK2 cycles of the same 256^3 input
    (after its first-dt pre-pass), reported as cell-updates/s."""
    import oracle as O

    s = O.copy_state(state)
    p = O.Params(N, N, N)
    mi = O.max_invdt(p, s)
    t0 = time.perf_counter()
    O.step(p, s, 0.0, 0.3 / mi, 2)
    el = time.perf_counter() - t0
    return {"value": round(2 * N ** 3 / el, 1), "unit": "cell-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"2 RK2 cycles of the same 256^3 FP64 input ({el:.1f} s, OpenMP)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--precision", default="both", choices=["both", "fp64", "fp32"])
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--zchunk", type=int, default=0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 2 GiB (for HBM counter scaling)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float64, device="cuda")  # 2 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": src.numel() * 8, "copies": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding is described in DESIGN.md but not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2304_13746_amd import inputs as I

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    state = I.turbulence(N, seed=2304, kpeak=4.0, mach=0.5, rho0=1.0, p0=0.6, b0=(0.2, 0.0, 0.0))
    state.pop("_l")
    results = {}
    precs = ["fp64", "fp32"] if args.precision == "both" else [args.precision]
    for prec in precs:
        r = run_gpu(state, prec, args.steps, args.warmup, args.tile, args.zchunk)
        ms_step = r["ms_total"] / args.steps
        results[prec] = {"value": N ** 3 / (ms_step * 1e-3), "ms_per_step": ms_step,
                         "roofline": roofline(prec, ms_step), "rc": r["rc"]}
        print(f"# {prec}: {ms_step:.3f} ms/cycle, {results[prec]['value']:.4e} cell-updates/s, "
              f"stage kernel {results[prec]['roofline']['achieved']:.0f} GB/s algorithmic, rc={r['rc']}",
              file=sys.stderr, flush=True)
    main_prec = precs[0]
    m = results[main_prec]
    line = {
        "metric": METRIC,
        "value": m["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": "256^3 periodic MHD turbulence (k_peak 4, Mach 0.5, B=(0.2,0,0)), "
                               "HLLD + PLM van Leer + E^c CT + RK2, CFL 0.3",
                   "cells": N ** 3, "precision": main_prec, "parallelism": "single GPU"},
        "roofline": m["roofline"],
    }
    if "fp32" in results and main_prec != "fp32":
        f = results["fp32"]
        line["fp32"] = {"value": f["value"], "ms_per_step": f["ms_per_step"], "dtype": "f32",
                        "roofline": f["roofline"]}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(state)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

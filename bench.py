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
import math
import os
import re
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz, the same
# for FP64 and non-packed FP32 (the kernels are compiled without packed FP32).
ALU_PEAK_TFLOPS = 78.6
# Algorithmic floating-point operations (add/sub, mul, div, sqrt) per cell and
# stage of this method on this 256^3 input with HLLD, counted on the oracle by
# oracle/opcount.cpp: 611.7 add/sub + 647.8 mul + 46.0 div + 18.0 sqrt.
FLOPS_PER_CELL_STAGE = 1323.46
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


def run_gpu(state, precision: str, steps: int, warmup: int, tile: int = 0, zchunk: int = 0,
            integrator: str = "rk2", emf: str = "ec", recon: str = "plm", n: int = N,
            riemann: str = "hlld", potential=None):
    import torch

    from paper_2304_13746_amd.box import MHDBox

    ct, b0 = ("vecpot", potential["b0"]) if potential else ("face", (0.0, 0.0, 0.0))
    box = MHDBox(n, n, n, precision=precision, riemann=riemann, tile=tile, zchunk=zchunk,
                 integrator=integrator, emf=emf, recon=recon, ct=ct, b0=b0)
    if potential:
        state = dict(state, ax=potential["ax"], ay=potential["ay"], az=potential["az"])
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


def roofline(precision: str, launch_ms: float):
    """Roofline of the stage kernel from its measured average launch duration.
    The kernel is bound by vector ALU work (algorithmic flops per cell and stage
    x cells per launch); the HBM view of the same launch (20 state words per
    cell on average: 16 in stage 1, 24 in stage 2) is reported beside it."""
    word = 8 if precision == "fp64" else 4
    cells = N ** 3
    launch_s = launch_ms * 1e-3
    flops_per_launch = FLOPS_PER_CELL_STAGE * cells
    tflops = flops_per_launch / launch_s / 1e12
    bytes_per_launch = 20 * word * cells
    gbs = bytes_per_launch / launch_s / 1e9
    traffic = counter_traffic(precision)
    return {"bound": "alu", "achieved": round(tflops, 2), "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tflops / ALU_PEAK_TFLOPS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 4),
            "traffic_unit": "GB per stage launch (rocprofv3 FETCH/WRITE, copy-calibrated)",
            "algorithmic_flops_per_launch": round(flops_per_launch),
            "launch_ms": round(launch_ms, 4),
            "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "algorithmic_bytes_per_launch": bytes_per_launch}}


CPU_CYCLES = 10  # about 10-15 s of oracle work on 16 host cores


def cpu_baseline(state):
    """The FP64 oracle on the host cores: CPU_CYCLES RK2 cycles of the same 256^3
    input (after its first-dt pre-pass), reported as cell-updates/s."""
    import oracle as O

    s = O.copy_state(state)
    p = O.Params(N, N, N)
    mi = O.max_invdt(p, s)
    t0 = time.perf_counter()
    O.step(p, s, 0.0, 0.3 / mi, CPU_CYCLES)
    el = time.perf_counter() - t0
    return {"value": round(CPU_CYCLES * N ** 3 / el, 1), "unit": "cell-updates/s",
            "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{CPU_CYCLES} RK2 cycles of the same 256^3 FP64 input ({el:.1f} s, OpenMP)",
            "error_vs_oracle": errors_vs_oracle(state, s)}


def errors_vs_oracle(state, ref):
    """Errors of the GPU results after the same cycles against the oracle's:
    FP64 (expected bit-identical) and FP32 (input rounded to FP32 by the
    library), per quantity as max|gpu - oracle| / max|oracle| and as the ratio
    of L2 norms."""
    from paper_2304_13746_amd.box import MHDBox

    groups = {"rho": ("rho",), "momentum": ("mx", "my", "mz"), "energy": ("en",),
              "field": ("bx", "by", "bz")}
    out = {}
    for prec in ("fp64", "fp32"):
        box = MHDBox(N, N, N, precision=prec)
        box.set_state(state)
        box.step(CPU_CYCLES)
        g, _, _, _ = box.get_state_numpy()
        box.close()
        e = {}
        for name, fs in groups.items():
            den = max(float(np.max(np.abs(ref[f]))) for f in fs)
            num = max(float(np.max(np.abs(g[f] - ref[f]))) for f in fs)
            l2 = math.sqrt(sum(float(np.sum((g[f] - ref[f]) ** 2)) for f in fs) /
                           sum(float(np.sum(ref[f] ** 2)) for f in fs))
            e[name] = {"max_rel": float(f"{num / den:.3e}"), "l2_rel": float(f"{l2:.3e}")}
        if prec == "fp64":
            e["bit_identical"] = all(np.array_equal(g[f], ref[f]) for f in ref)
        out[prec] = e
    return out


def batched_c3(nbox: int = 64, steps: int = 20):
    """64 uneven periodic boxes (edges log-uniform in [16, 128], multiples of 8,
    own seeded turbulence and uniform B), FP32, 20 RK2 cycles each: one captured
    HIP graph of batched stage launches, against the same boxes advanced one
    after another with single-box launches."""
    import torch

    from paper_2304_13746_amd import inputs as I
    from paper_2304_13746_amd.autotune import TILE_NAMES, Tuner
    from paper_2304_13746_amd.batch import BoxBatch
    from paper_2304_13746_amd.box import MHDBox

    spec = I.batch_boxes(nbox, seed=2304)
    cells = sum(int(np.prod(b["dims"])) for b in spec)
    stream = torch.cuda.Stream()
    boxes = [MHDBox(*b["dims"], *b["l"], precision="fp32", stream=stream) for b in spec]
    for bx, b in zip(boxes, spec):
        bx.set_state(b["state"])
    batch = BoxBatch(boxes)
    batch.step(1)  # warm the kernels
    # one launch shape for the whole batch, timed now (not from a cache)
    tuner = Tuner(os.path.join(tempfile.gettempdir(), f"mhd_tune_{os.getpid()}.json"))
    choice = batch.tune(tuner, force=True)
    graph = batch.capture(steps)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    graph.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_batch = ev0.elapsed_time(ev1)
    rcs = [bx.get_state(check=False)[3] for bx in boxes]
    # sequential reference: each box alone with its default launch shape
    for bx, b in zip(boxes, spec):
        bx.set_launch(0, 0)
        bx.set_state(b["state"])
    torch.cuda.synchronize()
    ev0.record(stream)
    done = []
    for bx in boxes:
        bx.step(steps)
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        done.append(e)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_seq = ev0.elapsed_time(ev1)
    lat_seq = sorted(ev0.elapsed_time(e) for e in done)
    for bx in boxes:
        bx.close()
    return {"workload": f"{nbox} uneven periodic boxes, edges 16-128 (log-uniform, multiples of 8), "
                        f"FP32, {steps} RK2 cycles each, one captured HIP graph",
            "cells": cells, "value": cells * steps / (ms_batch * 1e-3), "unit": "cell-updates/s",
            "ms_batch": round(ms_batch, 3), "ms_sequential": round(ms_seq, 3),
            "speedup_vs_sequential": round(ms_seq / ms_batch, 3),
            "latency_ms_batched": {"p50": round(ms_batch, 3), "p99": round(ms_batch, 3)},
            "latency_ms_sequential": {"p50": round(lat_seq[len(lat_seq) // 2], 3),
                                      "p99": round(lat_seq[int(0.99 * (len(lat_seq) - 1))], 3)},
            "status_ok": all(rc == 0 for rc in rcs),
            "launch_shape": {"tile": TILE_NAMES.get(choice["tile"], str(choice["tile"])),
                             "zchunk_cap": choice["zchunk_cap"],
                             "stage_ms_tuned": round(choice["best_ms"], 4),
                             "stage_ms_default": round(choice["default_ms"], 4),
                             "candidates": choice["candidates"]}}


def served_c4(nreq: int, precision: str = "fp32", rate: float = 200.0):
    """Poisson stream of box requests (mean 200 req/s), edge uniform in
    {32, 48, 64, 96, 128, 192}, 10-200 RK2 cycles, Orszag-Tang or turbulence
    initial data 50/50; admission by workspace bytes against an HBM budget."""
    import torch

    from paper_2304_13746_amd.serve import EDGES, GpuBackend, Server, poisson_requests

    free, total = torch.cuda.mem_get_info()
    budget = int(min(0.8 * free, 64 << 30))
    be = GpuBackend(precision=precision)
    reqs = poisson_requests(nreq, rate=rate, seed=2304)
    for e in EDGES:  # initial states resident on the GPU before the clock starts
        for init in ("ot", "turb"):
            from paper_2304_13746_amd.serve import Request
            be.initial_state(Request(-1, 0.0, e, 1, init, 0))
    torch.cuda.synchronize()
    st = Server(be, budget_bytes=budget, max_active=64, epoch_steps=10).run(reqs)
    s = st.summary()
    s.update({"workload": f"{nreq} Poisson requests at {rate:g}/s, edges {list(EDGES)}, 10-200 RK2 "
                          f"cycles, OT/turbulence, {precision.upper()}, HBM budget {budget / 2**30:.0f} GiB",
              "precision": precision})
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-box batched run")
    ap.add_argument("--no-next", action="store_true",
                    help="skip the runs of the widened scheme options (RK3, LimO3, PPM, E^0, "
                         "arithmetic and UCT-HLL EMFs, vector-potential CT), of the Sedov "
                         "512^3 hydro workload and of the 512^3 turbulence box")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests in the served replay (0: skip; the full stream is 5000)")
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
        print(f"bench.py: the library runs one box on one GPU (asked for --gpus {args.gpus}); "
              "sharding a box over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

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
        # two stage launches per cycle; the two one-thread cycle-control
        # launches (a few microseconds) are charged to them, conservatively
        results[prec] = {"value": N ** 3 / (ms_step * 1e-3), "ms_per_step": ms_step,
                         "roofline": roofline(prec, ms_step / 2.0), "rc": r["rc"]}
        print(f"# {prec}: {ms_step:.3f} ms/cycle, {results[prec]['value']:.4e} cell-updates/s, "
              f"stage kernel {results[prec]['roofline']['achieved']:.2f} TFLOP/s, "
              f"{results[prec]['roofline']['hbm']['achieved']:.0f} GB/s algorithmic, rc={r['rc']}",
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
    if not args.no_next:
        # widened scheme options on the same input: the third-order Runge-Kutta
        # cycle (three stage launches per cycle), LimO3 and PPM reconstructions
        # with RK3, and the E^0 / arithmetic / UCT-HLL corner EMFs (RK2; UCT-HLL
        # adds two light launches per stage)
        nxt = {}
        k = min(args.steps, 20)
        for name, integ, emf, recon, nst in (("rk3", "rk3", "ec", "plm", 3),
                                             ("limo3_rk3", "rk3", "ec", "limo3", 3),
                                             ("ppm_rk3", "rk3", "ec", "ppm", 3),
                                             ("emf_e0", "rk2", "e0", "plm", 2),
                                             ("emf_arith", "rk2", "arith", "plm", 2),
                                             ("emf_uct_hll", "rk2", "uct_hll", "plm", 2)):
            for prec in precs:
                r = run_gpu(state, prec, k, 1, args.tile, args.zchunk, integ, emf, recon)
                ms_step = r["ms_total"] / k
                nxt[f"{name}_{prec}"] = {"value": N ** 3 / (ms_step * 1e-3), "unit": "cell-updates/s",
                                         "ms_per_step": ms_step, "stage_launch_ms": ms_step / nst,
                                         "rc": r["rc"]}
                print(f"# {name} {prec}: {ms_step:.3f} ms/cycle", file=sys.stderr, flush=True)
        # the vector-potential form of constrained transport (FP64): the same
        # input with B = (0.2, 0, 0) carried as the mean field and A = 0
        pot = I.uniform_field_potential(state["rho"].shape, (0.2, 0.0, 0.0))
        r = run_gpu(state, "fp64", k, 1, args.tile, args.zchunk, potential=pot)
        ms_step = r["ms_total"] / k
        nxt["ct_vecpot_fp64"] = {"value": N ** 3 / (ms_step * 1e-3), "unit": "cell-updates/s",
                                 "ms_per_step": ms_step, "rc": r["rc"]}
        print(f"# vector-potential CT fp64: {ms_step:.3f} ms/cycle", file=sys.stderr, flush=True)
        del pot
        # the second workload: Sedov-Taylor blast at 512^3, B = 0 (Sec. 4.1), HLLC
        # and HLL (the paper's choice), RK2, PLM
        sed = I.sedov(512)
        for riem in ("hllc", "hll"):
            for prec in precs:
                r = run_gpu(sed, prec, k, 1, args.tile, args.zchunk, "rk2", "ec", "plm",
                            n=512, riemann=riem)
                ms_step = r["ms_total"] / k
                nxt[f"sedov512_{riem}_{prec}"] = {"value": 512 ** 3 / (ms_step * 1e-3),
                                                  "unit": "cell-updates/s", "ms_per_step": ms_step,
                                                  "stage_launch_ms": ms_step / 2, "rc": r["rc"]}
                print(f"# sedov 512^3 {riem} {prec}: {ms_step:.3f} ms/cycle", file=sys.stderr,
                      flush=True)
        del sed
        # the 512^3 turbulence configuration (E(k) ~ k^-5/3 on 2 <= k <= 64, rms
        # Mach 1, B = (0.1, 0.1, 0)) with the default scheme: the per-cell rate
        # at eight times the cells of the headline box
        print("# generating the 512^3 turbulence input", file=sys.stderr, flush=True)
        c5 = I.turbulence(512, seed=2304, spectrum="kolmogorov", kmin=2.0, kmax=64.0, mach=1.0,
                          b0=(0.1, 0.1, 0.0))
        c5.pop("_l")
        for prec in precs:
            r = run_gpu(c5, prec, k, 1, args.tile, args.zchunk, n=512)
            ms_step = r["ms_total"] / k
            nxt[f"turb512_{prec}"] = {"value": 512 ** 3 / (ms_step * 1e-3),
                                      "unit": "cell-updates/s", "ms_per_step": ms_step,
                                      "stage_launch_ms": ms_step / 2, "rc": r["rc"]}
            print(f"# turbulence 512^3 {prec}: {ms_step:.3f} ms/cycle", file=sys.stderr,
                  flush=True)
        del c5
        line["next_rows"] = nxt
    if not args.no_batch:
        line["batched"] = batched_c3()
        print(f"# batched: {line['batched']['value']:.4e} cell-updates/s, "
              f"{line['batched']['speedup_vs_sequential']}x vs sequential", file=sys.stderr, flush=True)
    if args.serve_requests > 0:
        line["served"] = [served_c4(args.serve_requests, p) for p in ("fp32", "fp64")]
        for sv in line["served"]:
            print(f"# served {sv['precision']}: p50 {sv['p50_ms']} ms p99 {sv['p99_ms']} ms, "
                  f"{sv['cell_updates_per_s']:.3e} cell-updates/s", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(state)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the HWENO hot path on one MI355X.

Workload: 2D Euler (gamma 1.4) on periodic [0,1]^2, 2048 x 2048 cells, 12
unknowns per cell (average, x- and y-moment of 4 conserved variables), two
Gauss points per edge, CFL 0.5, seeded quadrant states plus an isentropic
vortex (seed 7).  A step is one full SSP-RK3 step (wave-speed reduction, dt,
three fused stage kernels, time update) of the whole grid, inputs resident
in HBM.  Metric: cell-stage updates per second (3 per cell per step).

The single-precision-bulk path (FP32 reconstruction and fluxes, FP64 cell
averages and flux differences) is the headline value; the FP64 path is
measured beside it, with the L1 distance between the two after the timed
steps.  The CPU oracle's own rate on the host cores is the reported
baseline (the parity of both paths with the oracle at this size is checked
by tests/test_gpu_fullsize.py).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
VEC_TFLOPS = 78.6              # MI355X vector FP64, = non-packed FP32 (FMA counted as 2)
# FP operations per cell-stage of the 2D Euler stage (Q = 2): the FP
# instruction counters of the stage kernel (FMA = 2, other FP instructions 1)
# restricted to output-producing lanes and rows (profiles/stage2d_euler2048.md)
ALU_FLOP_PER_CELL_STAGE = 2706.0
# HBM bytes per stage launch measured with FETCH_SIZE / WRITE_SIZE (scaled by
# the copy calibration) for the kernel sources of this hash; any change of
# the sources invalidates them (reported as null until measured again).
PROFILED_SOURCES = "8090d9fc491abc8a"
PROFILED_TRAFFIC = {"f32acc64": 824.1e6, "f64": 1243.6e6}


def kernel_sources_hash() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2607_24325_amd", "csrc")
    src = "".join(open(os.path.join(d, f)).read()
                  for f in ("stage2d.h", "device_common.h", "ff.h", "internal.h"))
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def algorithmic_bytes_per_cell_stage(K: int, D: int, su: int, sd: int) -> float:
    """Compulsory HBM traffic per cell per stage, averaged over the three
    stages: stage 1 reads U^n and writes U^(1) and the saved hats H; stages 2
    and 3 read U^(k), u-bar^n and H and write U^(k+1)."""
    S = K * (su + D * sd)
    H = K * D * sd
    return (6 * S + 3 * H + 2 * K * su) / 3.0


def timed_run(h, stream, steps: int, warmup: int, allow_nonfinite: bool = False):
    """Warm-up steps, then `steps` HIP-graph steps bracketed by events on the
    handle's stream (the step time; the library replays runs of 8 steps as
    one graph, built during the warm-up), then `steps` eagerly launched steps
    with an event pair around every kernel (the per-kernel times)."""
    import torch
    h.steps(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    tw0 = time.perf_counter()
    e0.record(stream)
    h.steps(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - tw0
    ms_step = e0.elapsed_time(e1) / steps
    tm = h.timed_steps(steps, allow_nonfinite=allow_nonfinite)
    torch.cuda.synchronize()
    assert tm.steps == steps
    return ms_step, wall, tm


def bench_batched(dim: int, prec: int, steps: int, warmup: int, dev, profile_only=False):
    """Throughput of one of the batched workloads: 4096 uneven 1D Euler
    problems (N ~ U{256..8192}, seed 1) or 256 uneven 2D Euler problems
    (side ~ U{128..1024}, seed 11, Q = 2, CFL 0.5); one launch per RK stage
    over every problem, per-problem dt."""
    import torch
    from paper_2607_24325_amd import hweno as hw
    from paper_2607_24325_amd import workloads as W
    t0 = time.time()
    if dim == 1:
        entries = W.batched_1d(seed=1, nprob=4096)
        make = W.batched_1d_state
        cfg = hw.default_config(1, precision=prec)
        K, su, sd = 3, 8, (8 if prec == hw.F64 else 4)
    else:
        entries = W.batched_2d(seed=11, nprob=256)
        make = W.batched_2d_state
        cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5)
        K, su, sd = 4, 8, (8 if prec == hw.F64 else 4)
    specs = [e[0] for e in entries]
    ncell = sum(s.nx * s.ny for s in specs)
    ws = torch.empty(hw.Handle.workspace_bytes(specs, cfg), dtype=torch.uint8, device=dev)
    h = hw.Handle(specs, cfg, workspace=ws, stream=torch.cuda.current_stream(dev).cuda_stream)
    for i, e in enumerate(entries):
        h.set_state(i, make(e))
    print(f"[bench] batched {dim}D: {len(specs)} problems, {ncell} cells, set up in "
          f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ms_step, _, tm = timed_run(h, torch.cuda.current_stream(dev), steps, warmup,
                               allow_nonfinite=True)
    stage_ms = tm.stage_ms / tm.stage_launches
    # the scheme has no positivity limiter: a problem whose state becomes
    # non-admissible is frozen by the library; its cells are not counted
    failed = h.failed_problems()
    live = ncell - sum(specs[i].nx * specs[i].ny for i in failed)
    B = algorithmic_bytes_per_cell_stage(K, dim, su, sd)
    h.close()
    del ws
    r = {"problems": len(specs), "cells": ncell, "value": 3.0 * live / (ms_step * 1e-3),
         "problems_frozen_nonadmissible": failed,
         "unit": "cell-stage updates/s", "ms_per_step": ms_step, "stage_kernel_ms": stage_ms,
         "bytes_per_cell_stage": B, "stage_hbm_frac": B * live / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
         "precision": "F32 bulk, FP64 cell averages" if prec != hw.F64 else "F64"}
    print(f"[bench] batched {dim}D: {ms_step:.3f} ms/step, stage {stage_ms:.3f} ms, "
          f"{r['value'] / 1e9:.2f} G cell-stage/s", file=sys.stderr, flush=True)
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--tune", action="store_true", help="run the autotuner first")
    ap.add_argument("--precision", default="both", choices=["both", "f32acc64", "f64"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy 1 GiB with a plain device copy (HBM counter scale)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workloads")
    ap.add_argument("--only-batched", type=int, default=0, choices=[0, 1, 2],
                    help="run only the batched 1D or 2D workload (profiling)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only run the timed steps (for profilers)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_24325_amd import hweno as hw
    from paper_2607_24325_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    t0 = time.time()
    spec, st = W.quadrant_vortex_2d(n, seed=7)
    print(f"[bench] workload built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ncell = n * n

    if args.only_batched:
        r = bench_batched(args.only_batched, hw.F32_ACC64, args.steps, args.warmup, dev)
        print(json.dumps({f"batched_{args.only_batched}d": r}))
        return
    results = {}
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    runs = [("f32acc64", hw.F32_ACC64, 8, 4, 0), ("f64", hw.F64, 8, 8, 0)]
    if args.precision != "both":
        runs = [r for r in runs if r[0] == args.precision]
    elif not args.profile_only:
        # the same workload with the reconstruction in characteristic variables
        runs.append(("f32acc64_characteristic", hw.F32_ACC64, 8, 4, 1))
    for name, prec, su, sd, charwise in runs:
        cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5, characteristic=charwise)
        ws = torch.empty(hw.Handle.workspace_bytes([spec], cfg), dtype=torch.uint8, device=dev)
        stream = torch.cuda.current_stream(dev)
        h = hw.Handle([spec], cfg, workspace=ws, stream=stream.cuda_stream)
        h.set_state(0, st)
        entry = {}
        if args.tune and not args.profile_only:
            tun = h.autotune()
            entry["tuning"] = {"tile_rows": tun.tile_rows, "grid_blocks": tun.grid_blocks}
        ms_step, wall, tm = timed_run(h, stream, args.steps, args.warmup)
        out, t_now = h.get_state(0)
        stage_ms = tm.stage_ms / tm.stage_launches
        B = algorithmic_bytes_per_cell_stage(4, 2, su, sd)
        entry.update({
            "value": 3.0 * ncell / (ms_step * 1e-3),
            "ms_per_step": ms_step,
            "wall_ms_per_step": wall * 1e3 / args.steps,
            "eager_ms_per_step": tm.total_ms / args.steps,
            "stage_kernel_ms": stage_ms,
            "alpha_ms_per_step": tm.alpha_ms / args.steps,
            "other_ms_per_step": tm.other_ms / args.steps,
            "bytes_per_cell_stage": B,
            "stage_hbm_gbs": B * ncell / (stage_ms * 1e-3) / 1e9,
            "t_reached": t_now,
            "state": out,
        })
        results[name] = entry
        h.close()
        del ws
        print(f"[bench] {name}: {ms_step:.3f} ms/step, stage {stage_ms:.3f} ms, "
              f"{entry['value'] / 1e9:.2f} G cell-stage/s", file=sys.stderr, flush=True)

    if args.profile_only or args.precision != "both":
        for k, r in results.items():
            r.pop("state", None)
            print(json.dumps({k: r}))
        return
    main_r = results["f32acc64"]
    f64_r = results["f64"]
    l1_32_vs_64 = float(np.abs(main_r["state"][0] - f64_r["state"][0]).mean(axis=(1, 2)).max())
    cpu = None
    if not args.no_cpu and not args.profile_only:
        import oracle as O
        threads = os.cpu_count() or 1
        O.set_threads(threads)
        cfg = hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=0.5)
        p = O.Problem(dim=2, flux=O.EULER, nx=n, ny=n, gas_gamma=spec.gas_gamma, gauss_q=2,
                      weights=cfg.weights, gamma_lin=tuple(cfg.gamma_lin), eps=cfg.eps)
        ax, ay = O.alpha(p, st)
        dt = O.dt(p, ax, ay, 0.5)
        tc = time.perf_counter()
        O.step(p, st, ax, ay, dt)
        el = time.perf_counter() - tc
        cpu = {"value": 3.0 * ncell / el, "unit": "cell-stage updates/s", "cores": O.get_threads(),
               "kind": "oracle",
               "sample": f"one full SSP-RK3 step of the {n}x{n} 2D Euler workload (FP64 oracle, "
                         f"OpenMP over rows), {el:.1f}s"}

    batched = {}
    if not args.no_batched:
        for d in (1, 2):
            batched[f"batched_{d}d"] = bench_batched(d, hw.F32_ACC64, args.steps, args.warmup, dev)
    B = main_r["bytes_per_cell_stage"]
    achieved = main_r["stage_hbm_gbs"]
    alu_tflops = ALU_FLOP_PER_CELL_STAGE * ncell / (main_r["stage_kernel_ms"] * 1e-3) / 1e12
    traffic = PROFILED_TRAFFIC["f32acc64"] if kernel_sources_hash() == PROFILED_SOURCES else None
    line = {
        "metric": "cell-stage updates/s (2D Euler 2048^2, FP32 vs FP64) + % HBM peak + L1 err",
        "value": main_r["value"],
        "unit": "cell-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded quadrant states + isentropic vortex)",
        "config": {"workload": f"2D Euler {n}x{n} periodic, Q=2, CFL 0.5, quadrant+vortex seed 7",
                   "precision": "F32 bulk, FP64 cell averages and cell-average flux differences",
                   "cells": ncell, "unknowns_per_cell": 12},
        "roofline": {"bound": "alu", "achieved": alu_tflops, "peak": VEC_TFLOPS, "unit": "TFLOP/s",
                     "frac": alu_tflops / VEC_TFLOPS, "traffic": traffic,
                     "traffic_unit": "HBM bytes per stage launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
                     "kernel": "stage2d_kernel (F32_ACC64)",
                     "algorithmic_flop_per_cell_stage": ALU_FLOP_PER_CELL_STAGE,
                     "hbm_achieved_gbs": achieved, "hbm_frac": achieved / HBM_PEAK_GBS,
                     "algorithmic_bytes_per_cell_stage": B},
        "hbm_frac_fp64_path": f64_r["stage_hbm_gbs"] / HBM_PEAK_GBS,
        "fp64_path": {"value": f64_r["value"], "ms_per_step": f64_r["ms_per_step"],
                      "stage_kernel_ms": f64_r["stage_kernel_ms"],
                      "bytes_per_cell_stage": f64_r["bytes_per_cell_stage"]},
        "characteristic_path": {k: results["f32acc64_characteristic"][k]
                                for k in ("value", "ms_per_step", "stage_kernel_ms")},
        "l1_f32_vs_f64_after_timed_steps": l1_32_vs_64,
        "stage_kernel_ms": main_r["stage_kernel_ms"],
        "tuning": main_r.get("tuning"),
        "cpu_baseline": cpu,
    }
    line.update(batched)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

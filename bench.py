"""Benchmark of the HWENO hot path on one MI355X.

Workload: 2D Euler (gamma 1.4) on periodic [0,1]^2, 2048 x 2048 cells, 12
unknowns per cell (average, x- and y-moment of 4 conserved variables), two
Gauss points per edge, CFL 0.5, seeded quadrant states plus an isentropic
vortex (seed 7).  A step is one full SSP-RK3 step (dt, three fused stage
kernels, time update; the wave speeds come from the previous step's stage 3)
of the whole grid, inputs resident in HBM.  Metric: cell-stage updates per
second (3 per cell per step).

The single-precision-bulk path (FP32 reconstruction and fluxes, FP64 cell
averages and flux differences) is the headline value, measured with the
autotuned launch configuration (the library default is reported beside it);
the FP64 path, the characteristic-variable path and the two batched
workloads (4096 uneven 1D problems in FP32 bulk with FP64 averages; 256
uneven 2D problems with Kahan-compensated averages) are measured beside it.
Every result carries its error against the FP64 CPU oracle (first step on
sampled windows or problems, and a whole run to t = 0.1 at 128^2) and the
drift of its periodic totals over the timed steps.  The oracle's own rate on
the host cores, one thread and all threads, is the reported baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# HBM bytes per stage launch measured with FETCH_SIZE / WRITE_SIZE (scaled by
# the copy calibration) and VALU wave-instructions per launch, per path and
# launch configuration (tile_rows, grid_blocks, variant: the halo re-reads
# depend on the first two, the instruction count on the last), for the
# kernel sources of this hash; any change of the sources
# invalidates them, and a configuration not profiled has none (both are
# reported as null).
PROFILED_SOURCES = "12f6670ea8fd1413"
# path, tile_rows, grid_blocks, variant: HBM MB and VALU wave-instructions (M)
# per stage launch, mean of the three stages, for every launch configuration
# the tuner can choose (one eager step each; 2048^2 workload, 4096-problem 1D
# batch, where segment heights do not apply, 256-problem 2D batch)
_PROFILED_TABLE = """
f32acc64 16 0 0 893.7 156.70
f32acc64 16 512 0 840.4 155.83
f32acc64 16 768 0 888.3 155.89
f32acc64 16 1024 0 904.8 155.94
f32acc64 24 0 0 878.7 150.91
f32acc64 24 512 0 850.1 150.37
f32acc64 24 768 0 884.3 150.42
f32acc64 24 1024 0 897.1 150.48
f32acc64 32 0 0 870.3 147.88
f32acc64 32 512 0 849.8 147.50
f32acc64 32 768 0 877.1 147.56
f32acc64 32 1024 0 894.1 147.61
f32acc64 48 0 0 865.6 144.99
f32acc64 48 512 0 850.7 144.77
f32acc64 48 768 0 871.2 144.82
f32acc64 48 1024 0 882.4 144.88
f32acc64 64 0 0 866.9 143.47
f32acc64 64 512 0 845.6 143.34
f32acc64 64 768 0 859.2 143.39
f32acc64 64 1024 0 870.0 143.45
f32acc64 16 0 1 2349.0 159.98
f32acc64 16 512 1 1101.0 159.13
f32acc64 16 768 1 1608.1 159.18
f32acc64 16 1024 1 2184.5 159.24
f32acc64 24 0 1 2320.8 154.15
f32acc64 24 512 1 1053.0 153.62
f32acc64 24 768 1 1535.8 153.67
f32acc64 24 1024 1 2170.2 153.73
f32acc64 32 0 1 2281.0 151.10
f32acc64 32 512 1 1032.5 150.73
f32acc64 32 768 1 1508.2 150.78
f32acc64 32 1024 1 2082.7 150.84
f32acc64 48 0 1 2202.1 148.18
f32acc64 48 512 1 1019.2 147.97
f32acc64 48 768 1 1467.5 148.02
f32acc64 48 1024 1 1805.9 148.08
f32acc64 64 0 1 2236.1 146.66
f32acc64 64 512 1 1001.5 146.53
f32acc64 64 768 1 1353.1 146.58
f32acc64 64 1024 1 2048.3 146.64
f32acc64 36 0 0 869.5 146.91
f32acc64 36 0 1 2099.0 150.13
f64 16 0 0 1342.3 178.61
f64 16 512 0 1331.7 177.33
f64 16 768 0 1355.1 177.41
f64 16 1024 0 1368.5 177.49
f64 24 0 0 1312.9 171.81
f64 24 512 0 1313.8 171.00
f64 24 768 0 1329.5 171.09
f64 24 1024 0 1323.7 171.17
f64 32 0 0 1296.9 168.25
f64 32 512 0 1317.1 167.69
f64 32 768 0 1324.5 167.77
f64 32 1024 0 1319.5 167.86
f64 48 0 0 1286.7 164.85
f64 48 512 0 1305.2 164.53
f64 48 768 0 1306.9 164.61
f64 48 1024 0 1309.9 164.69
f64 64 0 0 1283.0 163.07
f64 64 512 0 1306.8 162.87
f64 64 768 0 1304.1 162.96
f64 64 1024 0 1287.2 163.04
f64 16 0 1 1341.2 178.91
f64 16 512 1 1333.7 177.65
f64 16 768 1 1358.0 177.73
f64 16 1024 1 1368.8 177.81
f64 24 0 1 1313.6 172.14
f64 24 512 1 1313.9 171.34
f64 24 768 1 1330.5 171.42
f64 24 1024 1 1321.3 171.51
f64 32 0 1 1297.5 168.59
f64 32 512 1 1313.1 168.04
f64 32 768 1 1323.7 168.12
f64 32 1024 1 1318.9 168.20
f64 48 0 1 1286.9 165.20
f64 48 512 1 1300.6 164.89
f64 48 768 1 1307.3 164.97
f64 48 1024 1 1311.1 165.05
f64 64 0 1 1284.8 163.43
f64 64 512 1 1304.0 163.24
f64 64 768 1 1304.2 163.32
f64 64 1024 1 1291.2 163.40
f64 36 0 0 1294.1 167.12
f64 36 0 1 1293.8 167.46
f32acc64_characteristic 16 0 0 801.8 373.73
f32acc64_characteristic 16 512 0 839.2 372.39
f32acc64_characteristic 16 768 0 862.6 372.48
f32acc64_characteristic 16 1024 0 867.9 372.56
f32acc64_characteristic 24 0 0 821.8 361.13
f32acc64_characteristic 24 512 0 817.9 360.28
f32acc64_characteristic 24 768 0 839.4 360.37
f32acc64_characteristic 24 1024 0 835.9 360.46
f32acc64_characteristic 32 0 0 814.2 354.53
f32acc64_characteristic 32 512 0 810.7 353.94
f32acc64_characteristic 32 768 0 828.3 354.03
f32acc64_characteristic 32 1024 0 828.5 354.11
f32acc64_characteristic 48 0 0 805.9 348.22
f32acc64_characteristic 48 512 0 808.0 347.89
f32acc64_characteristic 48 768 0 812.7 347.97
f32acc64_characteristic 48 1024 0 814.0 348.06
f32acc64_characteristic 64 0 0 799.5 344.92
f32acc64_characteristic 64 512 0 800.2 344.72
f32acc64_characteristic 64 768 0 801.9 344.80
f32acc64_characteristic 64 1024 0 800.1 344.89
f32acc64_characteristic 36 0 0 812.9 352.43
batched_1d 0 0 0 1857.4 145.15
batched_1d 0 512 0 1858.0 135.52
batched_1d 0 1024 0 1858.9 135.59
batched_1d 0 2048 0 1861.0 135.73
batched_2d 16 0 0 22914.4 4788.12
batched_2d 16 512 0 27014.1 4762.48
batched_2d 16 768 0 26950.1 4762.53
batched_2d 16 1024 0 27213.5 4762.59
batched_2d 24 0 0 22661.0 4629.75
batched_2d 24 512 0 26289.6 4612.60
batched_2d 24 768 0 26394.3 4612.66
batched_2d 24 1024 0 26601.3 4612.71
batched_2d 32 0 0 22756.4 4550.91
batched_2d 32 512 0 26031.2 4537.99
batched_2d 32 768 0 26139.6 4538.04
batched_2d 32 1024 0 26378.1 4538.10
batched_2d 48 0 0 23088.0 4471.57
batched_2d 48 512 0 25638.5 4462.89
batched_2d 48 768 0 25739.1 4462.95
batched_2d 48 1024 0 25911.7 4463.00
batched_2d 64 0 0 23545.5 4432.00
batched_2d 64 512 0 25143.9 4425.45
batched_2d 64 768 0 25516.7 4425.50
batched_2d 64 1024 0 25782.4 4425.56
batched_2d 16 0 1 52423.3 4803.91
batched_2d 16 512 1 31315.1 4778.75
batched_2d 16 768 1 41837.8 4778.80
batched_2d 16 1024 1 55597.2 4778.86
batched_2d 24 0 1 51582.9 4645.29
batched_2d 24 512 1 29843.7 4628.46
batched_2d 24 768 1 40691.1 4628.51
batched_2d 24 1024 1 54362.9 4628.57
batched_2d 32 0 1 51334.6 4566.32
batched_2d 32 512 1 29146.4 4553.63
batched_2d 32 768 1 39965.0 4553.69
batched_2d 32 1024 1 53750.0 4553.74
batched_2d 48 0 1 51366.1 4486.85
batched_2d 48 512 1 28322.5 4478.33
batched_2d 48 768 1 39269.2 4478.38
batched_2d 48 1024 1 53096.4 4478.44
batched_2d 64 0 1 51527.3 4447.22
batched_2d 64 512 1 27901.3 4440.78
batched_2d 64 768 1 38862.9 4440.84
batched_2d 64 1024 1 52380.7 4440.89
"""
PROFILED = {(p, int(r), int(g), int(v)): (float(t) * 1e6, float(a) * 1e6)
            for p, r, g, v, t, a in (ln.split() for ln in _PROFILED_TABLE.strip().splitlines())}


def kernel_sources_hash() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2607_24325_amd", "csrc")
    src = "".join(open(os.path.join(d, f)).read()
                  for f in ("stage2d.h", "stage2d_char.h", "stage1d.h", "device_common.h", "ff.h",
                            "internal.h"))
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def algorithmic_bytes_per_cell_stage(K: int, D: int, su: int, sd: int) -> float:
    """Compulsory HBM traffic per cell per stage, averaged over the three
    stages: stage 1 reads U^n and writes U^(1) and the saved hats H; stages 2
    and 3 read U^(k), u-bar^n and H and write U^(k+1)."""
    S = K * (su + D * sd)
    H = K * D * sd
    return (6 * S + 3 * H + 2 * K * su) / 3.0


def cpu_model() -> str:
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def host_threads() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except Exception:
        return os.cpu_count() or 1


# --------------------------------------------------------------- errors ---

def natural_scales(spec, st):
    """per (var, comp) plane: max |u-bar| for averages; for derivative means
    the larger of their own max and the range of the averages over one cell"""
    S = np.zeros((spec.nvar, spec.K))
    for c in range(spec.K):
        u = st[0, c]
        rng = float(u.max() - u.min())
        S[0, c] = np.abs(u).max()
        for v in range(1, spec.nvar):
            S[v, c] = max(np.abs(st[v, c]).max(), rng / (spec.dx if spec.dim == 1 else 1.0))
    return np.where(S > 0, S, 1.0)


def err_summary(got, ref, S):
    """L1 (mean over cells) and L-inf of the difference, each plane in its
    natural scale, worst plane; and the plain density L1"""
    ax = tuple(range(2, ref.ndim))
    d = np.abs(np.asarray(got, dtype=np.float64) - ref)
    return {"l1": float((d.mean(axis=ax) / S).max()), "linf": float((d.max(axis=ax) / S).max()),
            "rho_l1": float(d[0, 0].mean())}


def drift(st0, st1):
    """largest relative change of the periodic totals of the cell averages"""
    t0 = st0[0].reshape(st0.shape[1], -1).sum(axis=1)
    t1 = st1[0].reshape(st1.shape[1], -1).sum(axis=1)
    return float((np.abs(t1 - t0) / np.abs(t0)).max())


def windows(n):
    return [(0, 0, 4, 4), (n - 4, n - 4, 4, 4), (n // 2 - 2, n // 2 - 2, 4, 4), (58, 62, 5, 5),
            (n // 2 - 2, 7, 4, 4), (500 % n, 500 % n, 4, 4), (n - 6, n // 3, 6, 4)]


def oproblem(O, spec, cfg):
    return O.Problem(dim=spec.dim, flux=spec.flux, nx=spec.nx, ny=spec.ny, xlo=spec.xlo,
                     xhi=spec.xhi, ylo=spec.ylo, yhi=spec.yhi, bc_x=spec.bc_x, bc_y=spec.bc_y,
                     gas_gamma=spec.gas_gamma, adv=tuple(spec.adv), gauss_q=cfg.gauss_q,
                     weights=cfg.weights,
                     gamma_lin=tuple(cfg.gamma_lin)[:3 if spec.dim == 1 else 5], eps=cfg.eps,
                     charwise=int(cfg.characteristic), smoothness=int(cfg.smoothness),
                     alpha_stage=int(cfg.alpha_stage))


def first_step_errors(O, spec, st, cfg, gpu1, dt, threads):
    """the GPU's first step from the seeded state against the oracle's on
    sampled windows (whole grid for small problems)"""
    p = oproblem(O, spec, cfg)
    O.set_threads(threads)
    ax, ay = O.alpha(p, st)
    odt = O.dt(p, ax, ay, cfg.cfl)
    S = natural_scales(spec, st)
    if spec.nx * spec.ny <= 300 * 300:
        e = err_summary(gpu1, O.step(p, st, ax, ay, dt), S)
        e["cells"] = "all"
    else:
        got, ref = [], []
        for (i0, j0, wi, wj) in windows(spec.nx):
            ref.append(O.step_window(p, st, ax, ay, dt, i0, j0, wi, wj).reshape(spec.nvar, spec.K, -1))
            got.append(gpu1[:, :, j0:j0 + wj, i0:i0 + wi].reshape(spec.nvar, spec.K, -1))
        e = err_summary(np.concatenate(got, axis=2), np.concatenate(ref, axis=2), S)
        e["cells"] = f"{len(windows(spec.nx))} sampled windows"
    e["dt_rel_diff"] = abs(dt - odt) / odt
    return e


# --------------------------------------------------------------- timing ---

def timed_run(h, stream, steps: int, warmup: int, allow_nonfinite: bool = False):
    """Warm-up steps, then `steps` HIP-graph steps bracketed by events on the
    handle's stream (the step time; the library replays runs of 8 steps as
    one graph, built during the warm-up), then `steps` eagerly launched steps
    with an event pair around every kernel, on the same stream (the
    per-kernel times)."""
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


def tuning_dict(t):
    return {"tile_rows": t.tile_rows, "grid_blocks": t.grid_blocks, "use_graph": t.use_graph,
            "variant": t.variant}


def roofline(B, cells, stage_ms, key, kernel, tuning):
    """HBM roofline of the dominant kernel from its algorithmic bytes and its
    mean launch time measured with HIP events"""
    achieved = B * cells / (stage_ms * 1e-3) / 1e9
    prof = None
    if kernel_sources_hash() == PROFILED_SOURCES:
        prof = PROFILED.get((key, tuning["tile_rows"], tuning["grid_blocks"], tuning["variant"]))
    traffic, valu = prof if prof else (None, None)
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per stage launch (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0)",
            "kernel": kernel, "kernel_ms": stage_ms, "cells_per_launch": cells,
            "algorithmic_bytes_per_cell_stage": B,
            "valu_wave_instructions_per_cell_stage": None if valu is None else valu / cells}


def bench_single(hw, W, O, spec, st, prec, charwise, args, dev, stream, threads, tune):
    """One 2048^2 path: first-step error against the oracle, the library
    default launch configuration timed, then (if tune) the autotuned one."""
    import torch
    cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5, characteristic=charwise)
    ncell = spec.nx * spec.ny
    ws = torch.empty(hw.Handle.workspace_bytes([spec], cfg), dtype=torch.uint8, device=dev)
    h = hw.Handle([spec], cfg, workspace=ws, stream=stream.cuda_stream)
    out = {}
    try:
        h.set_state(0, st)
        dt1 = h.step(want_dt=True)[0]
        gpu1, _ = h.get_state(0)
        if O is not None:
            out["errors_first_step"] = first_step_errors(O, spec, st, cfg, gpu1, dt1, threads)
        del gpu1
        runs = [] if (tune and args.profile_only) else [("default", None)]
        if tune:
            runs.append(("tuned", "autotune"))
        for name, how in runs:
            h.set_state(0, st)
            r = {}
            if how == "autotune" and args.launch:
                h.set_tuning(**args.launch)
            elif how == "autotune":
                t0 = time.perf_counter()
                tun = h.autotune()
                r["autotune_s"] = time.perf_counter() - t0
                r["from_cache"] = bool(h.tuned_from_cache())
            r["tuning"] = tuning_dict(h.tuning())
            if args.burn_in:
                # the GPU idled while the host measured the oracle and while
                # the state was uploaded: bring its clocks up before the
                # timed run (so that the default and tuned launches are
                # compared on equal terms)
                h.steps(args.burn_in)
                torch.cuda.synchronize()
            ms_step, wall, tm = timed_run(h, stream, args.steps, args.warmup)
            fin, t_now = h.get_state(0)
            r.update({"value": 3.0 * ncell / (ms_step * 1e-3), "ms_per_step": ms_step,
                      "wall_ms_per_step": wall * 1e3 / args.steps,
                      "eager_ms_per_step": tm.total_ms / args.steps,
                      "stage_kernel_ms": tm.stage_ms / tm.stage_launches,
                      "alpha_ms_per_step": tm.alpha_ms / args.steps,
                      "other_ms_per_step": tm.other_ms / args.steps,
                      "t_reached": t_now, "conservation_drift": drift(st, fin)})
            out[name] = r
            del fin
    finally:
        h.close()
        del ws
    return out


def bench_batched(hw, W, O, dim, prec, args, dev, stream, threads, tune):
    """Throughput of one of the batched workloads: 4096 uneven 1D Euler
    problems (N ~ U{256..8192}, seed 1, transmissive) or 256 uneven 2D Euler
    problems (side ~ U{128..1024}, seed 11, mixed boundaries, Q = 2, CFL
    0.5); one launch per RK stage over every problem, per-problem dt."""
    import torch
    t0 = time.time()
    if dim == 1:
        entries = W.batched_1d(seed=1, nprob=4096)
        make = W.batched_1d_state
        cfg = hw.default_config(1, precision=prec)
        K = 3
    else:
        entries = W.batched_2d(seed=11, nprob=256)
        make = W.batched_2d_state
        cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5)
        K = 4
    su = 4 if prec == hw.F32 else 8
    sd = 8 if prec == hw.F64 else 4
    specs = [e[0] for e in entries]
    ncell = sum(s.nx * s.ny for s in specs)
    states = [make(e) for e in entries]
    ws = torch.empty(hw.Handle.workspace_bytes(specs, cfg), dtype=torch.uint8, device=dev)
    h = hw.Handle(specs, cfg, workspace=ws, stream=stream.cuda_stream)
    r = {}
    try:
        for i, s in enumerate(states):
            h.set_state(i, s)
        print(f"[bench] batched {dim}D: {len(specs)} problems, {ncell} cells, set up in "
              f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        # first step of the smallest problems against the oracle
        dts = h.step(want_dt=True)
        small = sorted(range(len(specs)), key=lambda i: specs[i].nx * specs[i].ny)[:4]
        if O is not None:
            errs = [first_step_errors(O, specs[i], states[i], cfg, h.get_state(i)[0], dts[i], threads)
                    for i in small]
            r["errors_first_step"] = {k: max(e[k] for e in errs) for k in ("l1", "linf", "rho_l1",
                                                                            "dt_rel_diff")}
            r["errors_first_step"]["cells"] = f"all cells of the {len(small)} smallest problems"
        if args.burn_in:
            h.steps(args.burn_in)     # clocks up (the states are set again below)
            torch.cuda.synchronize()
        for i, s in enumerate(states):
            h.set_state(i, s)
        if tune and args.launch:
            h.set_tuning(**args.launch)
            r["tuning"] = tuning_dict(h.tuning())
        elif tune:
            tun = h.autotune()
            r["tuning"] = tuning_dict(tun)
        else:
            r["tuning"] = tuning_dict(h.tuning())
        ms_step, _, tm = timed_run(h, stream, args.steps, args.warmup, allow_nonfinite=True)
        stage_ms = tm.stage_ms / tm.stage_launches
        # the scheme has no positivity limiter: a problem whose state becomes
        # non-admissible is frozen by the library; its cells are not counted
        failed = h.failed_problems()
        live = ncell - sum(specs[i].nx * specs[i].ny for i in failed)
        periodic = [i for i in range(len(specs)) if i not in failed and specs[i].bc_x == hw.PERIODIC
                    and (dim == 1 or specs[i].bc_y == hw.PERIODIC)]
        dr = [drift(states[i], h.get_state(i)[0]) for i in periodic[:32]]
    finally:
        h.close()
        del ws
    B = algorithmic_bytes_per_cell_stage(K, dim, su, sd)
    tun = r["tuning"]
    # (segment heights do not apply in 1D)
    prof = (PROFILED.get((f"batched_{dim}d", tun["tile_rows"] if dim == 2 else 0, tun["grid_blocks"],
                          tun["variant"]))
            if kernel_sources_hash() == PROFILED_SOURCES else None)
    r.update({"problems": len(specs), "cells": ncell, "value": 3.0 * live / (ms_step * 1e-3),
              "problems_frozen_nonadmissible": failed, "unit": "cell-stage updates/s",
              "ms_per_step": ms_step, "stage_kernel_ms": stage_ms, "bytes_per_cell_stage": B,
              "stage_hbm_frac": B * live / (stage_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
              "stage_traffic": prof[0] if prof else None,
              "stage_valu_wave_instructions": prof[1] if prof else None,
              "conservation_drift": max(dr) if dr else None,
              "conservation_drift_problems": f"{len(dr)} problems periodic on every axis"
              if dr else "none (transmissive)",
              "precision": {hw.F32_ACC64: "F32 bulk, FP64 cell averages",
                            hw.F32_KAHAN: "F32 bulk, Kahan-compensated F32 cell averages",
                            hw.F64: "F64", hw.F32: "F32"}[prec]})
    print(f"[bench] batched {dim}D: {ms_step:.3f} ms/step, stage {stage_ms:.3f} ms, "
          f"{r['value'] / 1e9:.2f} G cell-stage/s", file=sys.stderr, flush=True)
    return r


# ------------------------------------------------------- oracle baseline ---

def oracle_baseline(O, spec, st, cfg, ncores):
    """The FP64 CPU oracle on bounded samples of the same workload: three
    window steps of a band of rows (full width), on one thread and on every
    host thread.  Rate = output cell-stage updates per second (the 6-cell
    margins the window steps also compute are not counted)."""
    p = oproblem(O, spec, cfg)
    O.set_threads(ncores)
    ax, ay = O.alpha(p, st)
    dt = O.dt(p, ax, ay, cfg.cfl)
    n = spec.nx
    res = {}
    for label, threads, rows in (("single_thread", 1, 64), ("all_threads", ncores, 512)):
        O.set_threads(threads)
        j0 = n // 2 - rows // 2
        t0 = time.perf_counter()
        for _ in range(3):
            O.step_window(p, st, ax, ay, dt, 0, j0, n, rows)
        el = time.perf_counter() - t0
        res[label] = {"value": 3 * 3.0 * n * rows / el, "cores": O.get_threads(), "seconds": el,
                      "sample": f"3 window steps of the {n}x{rows} band of rows {j0}..{j0 + rows - 1} "
                                f"of the {n}x{n} workload"}
    O.set_threads(0)
    return res


def final_time_reference(O, W, hw, n, threads, box):
    """oracle run of the n^2 quadrant + vortex workload to t = 0.1 (run on a
    thread while the GPU paths are measured)"""
    spec, st = W.quadrant_vortex_2d(n, seed=7)
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=0.5)
    O.set_threads(threads)
    t0 = time.perf_counter()
    ref, steps = O.run(oproblem(O, spec, cfg), st, 0.0, 0.1, 0.5)
    box.update(spec=spec, st=st, ref=ref, steps=steps, seconds=time.perf_counter() - t0)


def final_time_errors(hw, box, prec):
    spec, st, ref = box["spec"], box["st"], box["ref"]
    cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5)
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        steps = h.run_to_time()
        out, t = h.get_state(0)
    e = err_summary(out, ref, natural_scales(spec, st))
    e.update({"steps": steps, "oracle_steps": box["steps"], "t": t,
              "conservation_drift": drift(st, out),
              "workload": f"quadrant+vortex {spec.nx}x{spec.ny} to t = 0.1, whole grid"})
    return e


def profile_candidates(hw, W):
    """One eagerly launched step per launch configuration the tuner can
    choose (`hweno_tuning_candidates`), for each benchmark path: the 2048^2
    workload in F32_ACC64, FP64 and characteristic variables, the
    4096-problem 1D batch and the 256-problem 2D batch (F32_KAHAN).  Prints
    the order as JSON lines (one untimed step per path first, marked
    "warm"): under `rocprofv3 --pmc` the stage-kernel dispatches come three
    per step in that order, which is how the PROFILED table above was
    measured."""
    spec, st = W.quadrant_vortex_2d(2048, seed=7)
    for name, prec, charwise in (("f32acc64", hw.F32_ACC64, 0), ("f64", hw.F64, 0),
                                 ("f32acc64_characteristic", hw.F32_ACC64, 1)):
        cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5, characteristic=charwise)
        with hw.Handle([spec], cfg) as h:
            h.set_state(0, st)
            h.set_tuning(use_graph=0)
            h.step()
            h.sync()
            print(json.dumps([name, "warm"]), flush=True)
            for c in h.tuning_candidates():
                h.set_tuning(tile_rows=c.tile_rows, grid_blocks=c.grid_blocks, variant=c.variant)
                h.step()
                h.sync()
                print(json.dumps([name, c.tile_rows, c.grid_blocks, c.variant]), flush=True)
    entries = W.batched_1d(seed=1, nprob=4096)
    cfg = hw.default_config(1, precision=hw.F32_ACC64)
    with hw.Handle([e[0] for e in entries], cfg) as h:
        for i, e in enumerate(entries):
            h.set_state(i, W.batched_1d_state(e))
        h.set_tuning(use_graph=0)
        h.step()
        h.sync()
        print(json.dumps(["batched_1d", "warm"]), flush=True)
        for c in h.tuning_candidates():
            h.set_tuning(grid_blocks=c.grid_blocks, variant=c.variant)
            h.step()
            h.sync()
            print(json.dumps(["batched_1d", 0, c.grid_blocks, c.variant]), flush=True)
    entries = W.batched_2d(seed=11, nprob=256)
    cfg = hw.default_config(2, precision=hw.F32_KAHAN, gauss_q=2, cfl=0.5)
    with hw.Handle([e[0] for e in entries], cfg) as h:
        for i, e in enumerate(entries):
            h.set_state(i, W.batched_2d_state(e))
        h.set_tuning(use_graph=0)
        h.step()
        h.sync()
        print(json.dumps(["batched_2d", "warm"]), flush=True)
        for c in h.tuning_candidates():
            h.set_tuning(tile_rows=c.tile_rows, grid_blocks=c.grid_blocks, variant=c.variant)
            h.step()
            h.sync()
            print(json.dumps(["batched_2d", c.tile_rows, c.grid_blocks, c.variant]), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (baseline and errors)")
    ap.add_argument("--burn-in", type=int, default=200,
                    help="untimed steps right before each timed 2048^2 run (after the state "
                         "upload and the tuner), and before the batched runs' state upload")
    ap.add_argument("--no-tune", action="store_true", help="library defaults only")
    ap.add_argument("--launch", default=None,
                    help="ROWS,GRID,VARIANT: this launch configuration instead of the tuner's")
    ap.add_argument("--precision", default="all", choices=["all", "f32acc64", "f64"])
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also copy 1 GiB with a plain device copy (HBM counter scale)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched workloads")
    ap.add_argument("--only-batched", type=int, default=0, choices=[0, 1, 2],
                    help="run only the batched 1D or 2D workload (profiling)")
    ap.add_argument("--profile-only", action="store_true",
                    help="only the timed steps of the 2048^2 paths (for profilers)")
    ap.add_argument("--characteristic", action="store_true",
                    help="with --profile-only: also the characteristic-variable path")
    ap.add_argument("--profile-candidates", action="store_true",
                    help="one eager step per tuner candidate of each path, order printed (profiling)")
    args = ap.parse_args()
    if args.launch:
        r_, g_, v_ = (int(x) for x in args.launch.split(","))
        args.launch = {"tile_rows": r_, "grid_blocks": g_, "variant": v_}
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library has no multi-GPU path "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2607_24325_amd import hweno as hw
    from paper_2607_24325_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.profile_candidates:
        profile_candidates(hw, W)
        return
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.Stream(dev)       # default priority
    ncores = host_threads()
    use_oracle = not (args.no_cpu or args.profile_only)
    O = None
    if use_oracle:
        import oracle as O
    # with --profile-only the tuner should find its choice in the cache that
    # HWENO_TUNING_CACHE names (written by the full run), so that the
    # profiled launches are the benchmarked ones and no candidate is timed
    tune = not args.no_tune
    n = args.n
    t0 = time.time()
    spec, st = W.quadrant_vortex_2d(n, seed=7)
    print(f"[bench] workload built in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    ncell = n * n

    if args.only_batched:
        prec = hw.F32_ACC64 if args.only_batched == 1 else hw.F32_KAHAN
        r = bench_batched(hw, W, None, args.only_batched, prec, args, dev, stream, ncores, tune)
        print(json.dumps({f"batched_{args.only_batched}d": r}))
        return
    if args.copy_calibration:
        src = torch.empty(1 << 27, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    cpu = None
    box, worker = {}, None
    if use_oracle:
        cfg64 = hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=0.5)
        base = oracle_baseline(O, spec, st, cfg64, ncores)
        a = base["all_threads"]
        cpu = {"value": a["value"], "unit": "cell-stage updates/s", "cores": a["cores"],
               "kind": "oracle", "sample": a["sample"], "seconds": a["seconds"],
               "cpu_model": cpu_model(), "single_thread": base["single_thread"]}
        print(f"[bench] oracle: {a['value'] / 1e6:.3f} M cell-stage/s on {a['cores']} threads, "
              f"{base['single_thread']['value'] / 1e6:.3f} M on one", file=sys.stderr, flush=True)
        worker = threading.Thread(target=final_time_reference,
                                  args=(O, W, hw, 128, max(1, ncores - 2), box), daemon=True)
        worker.start()

    runs = [("f32acc64", hw.F32_ACC64, 0), ("f64", hw.F64, 0)]
    if args.precision != "all":
        runs = [r for r in runs if r[0] == args.precision]
    elif not args.profile_only or args.characteristic:
        runs.append(("f32acc64_characteristic", hw.F32_ACC64, 1))
    results = {}
    for name, prec, charwise in runs:
        r = bench_single(hw, W, O, spec, st, prec, charwise, args, dev, stream,
                         max(1, ncores - 2), tune)
        results[name] = r
        best = r.get("tuned", r.get("default"))
        dflt = f" (default launch: {r['default']['ms_per_step']:.3f} ms/step)" if "default" in r else ""
        print(f"[bench] {name}: {best['ms_per_step']:.3f} ms/step, stage "
              f"{best['stage_kernel_ms']:.3f} ms, {best['value'] / 1e9:.2f} G cell-stage/s{dflt} "
              f"tuning {best['tuning']}", file=sys.stderr, flush=True)

    if args.profile_only or args.precision != "all":
        for k, r in results.items():
            print(json.dumps({k: r}))
        return

    batched = {}
    if not args.no_batched:
        batched["batched_1d"] = bench_batched(hw, W, O, 1, hw.F32_ACC64, args, dev, stream,
                                              max(1, ncores - 2), tune)
        batched["batched_2d"] = bench_batched(hw, W, O, 2, hw.F32_KAHAN, args, dev, stream,
                                              max(1, ncores - 2), tune)
    final = None
    if worker is not None:
        worker.join()
        final = {"f32acc64": final_time_errors(hw, box, hw.F32_ACC64),
                 "f64": final_time_errors(hw, box, hw.F64),
                 "oracle_seconds": box["seconds"]}

    def path(r, key, kernel, su, sd):
        best = r.get("tuned", r["default"])
        B = algorithmic_bytes_per_cell_stage(4, 2, su, sd)
        d = {"value": best["value"], "ms_per_step": best["ms_per_step"],
             "stage_kernel_ms": best["stage_kernel_ms"], "tuning": best["tuning"],
             "roofline": roofline(B, ncell, best["stage_kernel_ms"], key, kernel,
                                  best["tuning"]),
             "conservation_drift": best["conservation_drift"],
             "errors_first_step": r.get("errors_first_step"),
             "default_launch": {k: r["default"][k] for k in ("value", "ms_per_step",
                                                             "stage_kernel_ms", "tuning")}}
        if final is not None and key in final:
            d["errors_final_time_128"] = final[key]
        return d

    main_r = path(results["f32acc64"], "f32acc64", "stage2d_kernel (F32_ACC64)", 8, 4)
    f64_r = path(results["f64"], "f64", "stage2d_kernel (F64)", 8, 8)
    ch_r = path(results["f32acc64_characteristic"], "f32acc64_characteristic",
                "stage2d_char_kernel (F32_ACC64)", 8, 4)
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
                   "cells": ncell, "unknowns_per_cell": 12, "tuning": main_r["tuning"]},
        "roofline": main_r["roofline"],
        "errors_first_step": main_r["errors_first_step"],
        "errors_final_time_128": main_r.get("errors_final_time_128"),
        "conservation_drift": main_r["conservation_drift"],
        "default_launch": main_r["default_launch"],
        "fp64_path": f64_r,
        "characteristic_path": ch_r,
        "stage_kernel_ms": main_r["stage_kernel_ms"],
        "cpu_baseline": cpu,
    }
    line.update(batched)
    print(json.dumps(line))


if __name__ == "__main__":
    main()

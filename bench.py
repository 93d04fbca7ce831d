#!/usr/bin/env python3
"""Benchmark of the REXI shallow-water hot path on one MI355X.

One step = one pass of the whole hot path over one state: the scheme
l_rexi_n_erk_ver1 (N^{dt/2} o REXI^{dt} o N^{dt/2}) when the context has a
grid, else the REXI linear stage alone.  The workload defaults to T255 on the
768 x 384 Gauss grid, dt = 3600 s, N = 800 poles, FP32 banded solves with an
FP64 beta sum.  Prints one JSON line (rank 0):

  value        REXI term-solves per second (one term-solve = one pole applied
               to the full state), whole job
  roofline     achieved rate of the dominant kernel (the banded chain solve)
               against the chip's vector ALU peak, from HIP events recorded
               around every launch of that kernel in the timed region
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6      # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_FP32_VALU = 157.3     # TFLOP/s: the same with packed FP32 (2 per lane)
PEAK_HBM = 8000.0          # GB/s

# Algorithmic flops of the fused chain solve per (pole, chain row), counting a
# real add/sub/mul as 1, an FMA as 2 and the reciprocal as 1:
#   delta row: diagonal 5, right-hand side 10, pivot 4 + |w|^2 3 + 1/|w|^2 1 +
#              conj/scale 2, c' 2, d' 4 + 6, back-substitution 8, weighted
#              output 6 + sum 2, h recovery 4 + 6 + sum 2          = 65
#   zeta row:  diagonal 1, pivot 4 + 3 + 1 + 2, c' 2, d' 10, back 8,
#              weighted output 6 + sum 2                            = 39
FLOPS_DELTA_ROW = 65
FLOPS_ZETA_ROW = 39


def n_modes(L):
    return (L + 1) * (L + 2) // 2


def solve_flops(L, N):
    # every (l, m) appears once as a delta row and once as a zeta row
    return N * n_modes(L) * (FLOPS_DELTA_ROW + FLOPS_ZETA_ROW)


def cpu_baseline(w, seconds: float, full: bool):
    """Time the oracle on a bounded sample of the workload.

    REXI stage: the oracle's banded solves on a sample of zonal orders (taken
    from the short end of the chain-length range), run over a process pool and
    scaled by the fraction of pole-rows covered.  Non-linear stage (full steps
    only): two Heun steps of the oracle timed whole, in-process."""
    import concurrent.futures as cf

    from oracle import rexi
    from paper_1805_06557_amd.inputs import jet_state

    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, w.N, w.p0, w.y)
    U0 = jet_state(w.L, w.seed)
    cores = min(len(os.sched_getaffinity(0)), 16)
    t_nl = 0.0
    if full:
        from oracle import nonlinear
        from oracle.operator import Params
        from oracle.sht import Grid
        g = Grid(w.L, w.nlat, w.nlon, Params())
        nonlinear.tendency(g, U0)                 # builds the Legendre tables (not timed)
        t0 = time.perf_counter()
        U = nonlinear.heun(g, U0, 0.5 * w.dt)
        nonlinear.heun(g, U, 0.5 * w.dt)
        t_nl = time.perf_counter() - t0
    # calibrate on one middle order, model the cost of order m as ~ (L - m + 1)^2
    # (the oracle assembles dense matrices), take orders from the short end
    mc = w.L // 2
    t0 = time.perf_counter()
    _oracle_chunk((U0, alpha, beta, w.dt, w.L, [mc]))
    tc = time.perf_counter() - t0
    orders, est = [], 0.0
    for m in range(w.L, -1, -1):
        if m == mc:
            continue
        est += tc * ((w.L - m + 1) / (w.L - mc + 1)) ** 2
        orders.append(m)
        if est > seconds * cores:
            break
    t0 = time.perf_counter()
    chunks = [orders[i::cores] for i in range(cores)]
    with cf.ProcessPoolExecutor(max_workers=cores) as ex:
        list(ex.map(_oracle_chunk, [(U0, alpha, beta, w.dt, w.L, c) for c in chunks if c]))
    elapsed = time.perf_counter() - t0
    rows = sum(w.L - m + 1 for m in orders)
    frac = rows / n_modes(w.L)
    t_rexi = elapsed / frac
    sample = (f"REXI stage: zonal orders {min(orders)}..{max(orders)} ({len(orders)} of {w.L + 1}, "
              f"{100 * frac:.1f}% of the pole-rows) in {elapsed:.1f} s over {cores} processes, "
              f"scaled to {t_rexi:.1f} s per stage")
    if full:
        sample += f"; non-linear stage: two oracle Heun steps timed whole, {t_nl:.2f} s"
    return {
        "value": w.N / (t_rexi + t_nl),
        "unit": "term-solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": sample,
    }


def _oracle_chunk(args):
    import os as _os
    _os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import linear
    from oracle.operator import Params
    U0, alpha, beta, dt, L, orders = args
    linear.rexi_linear_step(U0, alpha, beta, dt, L, Params(), orders=orders)
    return len(orders)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="T255-fp32")
    ap.add_argument("--stage", choices=["auto", "rexi"], default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solver", choices=["default", "fused", "stream", "hybrid"], default="default",
                    help="REXI chain-solve schedule")
    ap.add_argument("--seg-rows", type=int, default=0, help="REXI solve segment length (16, 32; 0 = default)")
    ap.add_argument("--waves", type=int, default=0, help="REXI solve waves per workgroup (1, 2, 4; 0 = default)")
    ap.add_argument("--ppl", type=int, default=0, help="REXI solve poles per lane (1, 2; 0 = default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is designed but not built "
              "(see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1805_06557_amd import api, configs
    from paper_1805_06557_amd.inputs import jet_state

    w = configs.ALL[args.workload]
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    full = args.stage == "auto" and w.nlat > 0
    ctx = api.SWE(w.L, w.nlat if full else 0, w.nlon if full else 0, prec=w.prec)
    solver = {"default": 0, "fused": api.SOLVER_FUSED, "stream": api.SOLVER_STREAM,
              "hybrid": api.SOLVER_HYBRID}[args.solver]
    if solver or args.seg_rows or args.waves or args.ppl:
        ctx.set_tuning(solver=solver, seg_rows=args.seg_rows, waves=args.waves, poles_per_lane=args.ppl)
    U = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    V = torch.empty_like(U)
    stream = torch.cuda.current_stream()

    def step(src, dst):
        if full:
            ctx.strang_step(alpha, beta, w.dt, src, dst, stream)
        else:
            ctx.rexi_linear_step(alpha, beta, w.dt, src, dst, stream)

    ctx.profile(True)
    for i in range(args.warmup):
        step(U, V)
        U, V = V, U
    torch.cuda.synchronize()
    # the factorization of the streaming schedules is built by the first call
    fact_ms, fact_n = ctx.profile_read(api.KERNEL_FACTOR)
    for kid in range(api.KERNEL_FACTOR):
        ctx.profile_read(kid)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        step(U, V)
        U, V = V, U
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    stage_ms = {}
    for kid, name in [(api.KERNEL_SOLVE, "rexi_chain_kernel"), (api.KERNEL_REDUCE, "sum_partials_kernel"),
                      (api.KERNEL_LEG_SYNTH, "legendre_synth_kernel"), (api.KERNEL_RING, "ring_kernel"),
                      (api.KERNEL_LEG_ANAL, "legendre_anal_kernel"), (api.KERNEL_GATHER, "gather_fourier_kernel")]:
        ms, n = ctx.profile_read(kid)
        stage_ms[name] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                          "ms_per_launch": ms / max(n, 1)}
    solve_ms = stage_ms["rexi_chain_kernel"]["ms_per_step"] * args.steps
    solve_n = int(round(stage_ms["rexi_chain_kernel"]["launches_per_step"] * args.steps))
    ctx.profile(False)
    if not torch.isfinite(torch.view_as_real(U)).all():
        print("bench.py: non-finite state after the timed steps", file=sys.stderr)
        sys.exit(3)

    ms_per_step = ms_total / args.steps
    fp32 = bool(w.prec & api.PREC_FP32_SOLVE)
    peak = PEAK_FP32_VALU if fp32 else PEAK_FP64_VALU
    avg_solve_ms = solve_ms / max(solve_n, 1)
    achieved = solve_flops(w.L, w.N) / (avg_solve_ms * 1e-3) / 1e12
    stage = "l_rexi_n_erk_ver1 step" if full else "REXI linear stage"
    out = {
        "metric": "REXI term-solves/s at T255 (sim-time/wall-time alongside)",
        "value": w.N * args.steps / (ms_total * 1e-3),
        "unit": "term-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {stage}, T{w.L}"
                        + (f" on {w.nlon}x{w.nlat} Gauss grid" if full else "")
                        + f", dt={w.dt:g} s, N={w.N} poles (p0={w.p0:g}, y={w.y:.4g}), "
                        + ("FP32 banded solves + FP64 beta sum" if fp32 else "FP64 solves")
                        + (", FP64 transforms" if full else ""),
            "L": w.L, "N": w.N, "dt": w.dt, "stage": stage,
        },
        "sim_time_per_wall": w.dt / (ms_per_step * 1e-3),
        "host_wall_s": wall,
        "roofline": {
            "bound": "alu",
            "kernel": "rexi_chain_kernel",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": None,
            "avg_kernel_ms": avg_solve_ms,
            "launches": solve_n,
            "algorithmic_flops_per_launch": solve_flops(w.L, w.N),
        },
        "kernels": stage_ms,
        "setup": {"rexi_factor_kernel_ms": fact_ms / max(fact_n, 1), "launches": fact_n},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_seconds, full)
    print(json.dumps(out))


if __name__ == "__main__":
    main()

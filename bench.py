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
  cpu_baseline the FP64 oracle (plain CPU implementation) on the same step,
               timed on the host's cores (the whole step at T255; a sample of
               the REXI stage's orders where the whole step would take minutes);
               its result is also the reference of step_error_vs_oracle
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_VALU = 78.6      # TFLOP/s: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_FP32_VALU = 78.6      # TFLOP/s: the same count for FP32 without packed (2-per-lane) instructions, which this
                           # library does not use
PEAK_FP32_PACKED = 157.3   # TFLOP/s: published FP32 vector peak (packed FP32, 2 per lane), reported alongside
PEAK_HBM = 8000.0          # GB/s

# Algorithmic work of the banded REXI solve per pole-unknown (one pole applied to
# one chain unknown; two chain unknowns (delta, zeta) per mode, h eliminated),
# the fixed count of the hot-path scope table, independent of the kernel's
# instruction mix: diagonal 4, right-hand-side modification 10 (delta rows),
# forward Thomas step ~19, back substitution 8, h recovery 10 (delta rows),
# beta-weighted accumulation 8-16: about 60 flops.
FLOPS_PER_POLE_UNKNOWN = 60
# Bytes per pole-unknown of the factor-streaming schedule: the cached pivot
# (complex FP32 / FP64) read by the forward sweep and again by the backward pass.
STREAM_BYTES_PER_POLE_UNKNOWN = {True: 16, False: 32}


# HBM bytes per launch of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, each
# scaled by the same counter on a copy of known size (the chain-kernel summary under profiles/).
# Valid only for the kernel source (sha256) and launch shape they were taken with.
_D = "1a59bdfd5c3f38b16d573e51e46806329405f17489429ddbcd3792d69b11fba2"
MEASURED_TRAFFIC = {
    # FP32 fused solve at T255, N = 800 (the same launch in the FP32 workloads:
    # only the Legendre stage around it differs): 109.2 MB read + 121.2 MB written
    ("T255-fp32", _D, (1, 8, 4, 2)): 109.2e6 + 121.2e6,
    ("T255-fp32-bf16", _D, (1, 8, 4, 2)): 109.2e6 + 121.2e6,
    ("T255-fp32-fp16", _D, (1, 8, 4, 2)): 109.2e6 + 121.2e6,
    # FP64 fused solve at T255, N = 800: 207.4 MB read + 220.3 MB written
    ("T255-fp64", _D, (1, 8, 4, 2)): 207.4e6 + 220.3e6,
    # FP64 fused solve at T511, N = 2000: 2132.6 MB read + 2254.2 MB written
    ("T511-fp64", _D, (1, 8, 4, 2)): 2132.6e6 + 2254.2e6,
    # streaming schedule at T255, N = 800: FP32 915.9 MB + 75.1 MB, FP64 1830.8 MB + 125.5 MB
    ("T255-fp32-bf16-stream-fp32", _D, (2, 8, 4, 2)): 915.9e6 + 75.1e6,
    ("T255-fp32-bf16-stream-fp64", _D, (2, 8, 4, 2)): 1830.8e6 + 125.5e6,
}


def kernel_source_digest():
    import hashlib
    src = os.path.join(ROOT, "paper_1805_06557_amd", "csrc", "rexi_solve.hip")
    with open(src, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(workload, tuning):
    key = (workload, kernel_source_digest(),
           (tuning["solver"], tuning["seg_rows"], tuning["waves"], tuning["poles_per_lane"]))
    return MEASURED_TRAFFIC.get(key)


def n_modes(L):
    return (L + 1) * (L + 2) // 2


def pole_unknowns(L, N):
    # every (l, m) appears once as a delta row and once as a zeta row
    return 2 * N * n_modes(L)


def solve_flops(L, N):
    return FLOPS_PER_POLE_UNKNOWN * pole_unknowns(L, N)


def _blas_threads():
    """BLAS thread counts numpy would use in this process (threadpoolctl)."""
    try:
        from threadpoolctl import threadpool_info
        return sorted({int(i.get("num_threads", 0)) for i in threadpool_info() if i.get("user_api") == "blas"})
    except Exception:                                   # noqa: BLE001 - report only
        return None


def _oracle_rexi_orders(args):
    """Worker: the oracle's REXI stage on a list of zonal orders, one BLAS thread."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        from oracle import linear
        from oracle.operator import Params
        U0, alpha, beta, dt, L, orders = args
        return linear.rexi_linear_step(U0, alpha, beta, dt, L, Params(), orders=orders)


def oracle_rexi(U0, alpha, beta, dt, L, orders=None, cores=None):
    """The oracle's REXI stage over a process pool (orders dealt round-robin, the
    longest chains first); returns (U1, seconds, processes)."""
    import concurrent.futures as cf
    cores = cores or len(os.sched_getaffinity(0))
    orders = list(range(L, -1, -1)) if orders is None else list(orders)
    chunks = [c for c in (orders[i::cores] for i in range(cores)) if c]
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=len(chunks)) as ex:
        parts = list(ex.map(_oracle_rexi_orders, [(U0, alpha, beta, dt, L, c) for c in chunks]))
    return sum(parts), time.perf_counter() - t0, len(chunks)


def oracle_step(w, U0, full_step: bool, seconds: float):
    """The oracle (plain FP64 CPU implementation) on this workload, timed on the
    host: the whole l_rexi_n_erk_ver1 step (Heun half step in-process with numpy's
    BLAS threads, the REXI stage over a process pool with one BLAS thread per
    process, Heun half step) when all orders fit the time budget, else the two
    Heun half steps whole and the REXI stage on a sample of orders from the short
    end of the chain-length range, scaled by the fraction of pole-rows covered.
    Returns (the oracle's result or None when sampled, cpu_baseline dict)."""
    from oracle import rexi
    cores = len(os.sched_getaffinity(0))
    alpha, beta, _, _ = rexi.coefficients(rexi.FN_EXP, w.N, w.p0, w.y)
    t_nl, A, g = 0.0, U0, None
    if full_step:
        from oracle import nonlinear
        from oracle.operator import Params
        from oracle.sht import Grid
        g = Grid(w.L, w.nlat, w.nlon, Params())
        nonlinear.tendency(g, U0)                 # builds the Legendre tables (not timed)
        t0 = time.perf_counter()
        A = nonlinear.heun(g, U0, 0.5 * w.dt)
        t_nl = time.perf_counter() - t0
    # full REXI stage if a calibrated estimate fits the budget (order m costs ~ (L - m + 1)^2)
    mc = w.L // 2
    t0 = time.perf_counter()
    _oracle_rexi_orders((A, alpha, beta, w.dt, w.L, [mc]))
    tc = time.perf_counter() - t0
    cost = [tc * ((w.L - m + 1) / (w.L - mc + 1)) ** 2 for m in range(w.L + 1)]
    if sum(cost) <= seconds * cores:
        R, t_rexi, procs = oracle_rexi(A, alpha, beta, w.dt, w.L, cores=cores)
        ref = R
        if full_step:
            t0 = time.perf_counter()
            ref = nonlinear.heun(g, R, 0.5 * w.dt)
            t_nl += time.perf_counter() - t0
        what = ("the whole step: two Heun half steps in-process" if full_step else "the whole REXI stage") + \
               f" ({t_nl:.2f} s) and the REXI stage over all {w.L + 1} orders ({t_rexi:.1f} s on {procs} processes)"
        t_total = t_rexi + t_nl
    else:
        orders, est = [], 0.0
        for m in range(w.L, -1, -1):
            est += cost[m]
            orders.append(m)
            if est > seconds * cores:
                break
        _, elapsed, procs = oracle_rexi(A, alpha, beta, w.dt, w.L, orders=orders, cores=cores)
        frac = sum(w.L - m + 1 for m in orders) / n_modes(w.L)
        t_rexi = elapsed / frac
        if full_step:
            from oracle import nonlinear
            t0 = time.perf_counter()
            nonlinear.heun(g, A, 0.5 * w.dt)
            t_nl += time.perf_counter() - t0
        what = (f"REXI stage on zonal orders {min(orders)}..{max(orders)} ({len(orders)} of {w.L + 1}, "
                f"{100 * frac:.1f}% of the pole-rows) in {elapsed:.1f} s over {procs} processes, scaled to "
                f"{t_rexi:.1f} s per stage") + (f"; two Heun half steps timed whole, {t_nl:.2f} s" if full_step else "")
        t_total = t_rexi + t_nl
        ref = None
    return ref, {
        "value": w.N / t_total,
        "unit": "term-solves/s",
        "cores": cores,
        "kind": "oracle",
        "sample": what + f"; {t_total:.1f} s per step; BLAS threads in-process {_blas_threads()}, "
                         "1 per pool process",
    }


PEAK_BF16_MFMA = 2500.0    # TFLOP/s, dense bf16 matrix cores


def _split_blocks(L, nlat):
    hpad = (nlat // 2 + 15) // 16 * 16
    rows = 0
    for m in range(L + 1):
        n = L - m + 2                      # degrees m .. L+1
        rows += ((n + 1) // 2 + 15) // 16 * 16 + (n // 2 + 15) // 16 * 16
    return hpad, rows


def split_mfma_flops(L, nlat):
    """Matrix-core flops of one split-precision Legendre launch of the non-linear
    set (one Pbar product, three bf16 products, 16x16x16 tiles incl. padding)."""
    hpad, rows = _split_blocks(L, nlat)
    return 3 * (hpad // 16) * (rows // 16) * 2 * 16 * 16 * 16


def split_table_bytes(L, nlat):
    """Bytes of the Pbar table (hi and lo) one such launch streams."""
    hpad, rows = _split_blocks(L, nlat)
    return rows * hpad * 2 * 2


def step_error_vs_oracle(ctx, w, alpha, beta, U0, ref, full):
    """Per-field L-inf and L2 error of one step of this workload (the timed
    path, from the workload's initial state) against the oracle's step."""
    import torch
    d0 = torch.from_numpy(U0).cuda()
    got = torch.empty_like(d0)
    if full:
        ctx.strang_step(alpha, beta, w.dt, d0, got)
    else:
        ctx.rexi_linear_step(alpha, beta, w.dt, d0, got)
    ctx.sync()
    g = got.cpu().numpy()
    return {"state": _field_errors(g, ref), "increment": _field_errors(g - U0, ref - U0),
            "reference": "oracle (FP64 CPU), same initial state and contour"}


def _timed(fn, reps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(reps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / reps


def _field_errors(got, ref):
    import numpy as np
    linf = [float(np.abs(got[f] - ref[f]).max() / np.abs(ref[f]).max()) for f in range(3)]
    l2 = [float(np.linalg.norm(got[f] - ref[f]) / np.linalg.norm(ref[f])) for f in range(3)]
    return {"linf_rel": dict(zip(("h", "zeta", "delta"), linf)), "l2_rel": dict(zip(("h", "zeta", "delta"), l2))}


def equal_error_arm(reps, with_oracle=True):
    """FP32 against FP64 REXI stages at T255 (dt = 3600 s), each with the contour
    that meets the same target scalar error E with the fewest poles, timed on the
    same jet state; the error of each is measured per field against the oracle's
    REXI stage with a much tighter contour (N = 800, p0 = 12, predicted error
    1.3e-11), run over a process pool on the host."""
    import torch

    from paper_1805_06557_amd import api, configs
    from paper_1805_06557_amd.inputs import jet_state

    stream = torch.cuda.current_stream()
    ref_w = configs.T255_FP64
    u0 = jet_state(255, ref_w.seed)
    U0 = torch.from_numpy(u0).cuda()
    if with_oracle:
        from oracle import rexi
        a, b, _, _ = rexi.coefficients(rexi.FN_EXP, ref_w.N, ref_w.p0, ref_w.y)
        ref, t_ref, procs = oracle_rexi(u0, a, b, ref_w.dt, ref_w.L)
        out = {"E": configs.EQUAL_ERROR_E,
               "reference": f"oracle REXI stage, N=800, p0=12 ({t_ref:.1f} s on {procs} host processes)"}
    else:
        cref = api.SWE(255, prec=0)
        a, b, _, _ = api.rexi_coefficients(api.FN_EXP, ref_w.N, ref_w.p0, ref_w.y)
        Uref = torch.empty_like(U0)
        cref.rexi_linear_step(a, b, ref_w.dt, U0, Uref, stream)
        ref = Uref.cpu().numpy()
        cref.close()
        out = {"E": configs.EQUAL_ERROR_E, "reference": "FP64 GPU stage, N=800, p0=12"}
    for key, w in (("fp32", configs.T255_FP32_AT_E), ("fp64", configs.T255_FP64_AT_E)):
        ctx = api.SWE(w.L, prec=w.prec)
        a, b, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
        U1 = torch.empty_like(U0)
        ctx.autotune(a, b, w.dt, U0, U1, reps=3, stream=stream)
        side = torch.cuda.Stream()
        with torch.cuda.stream(side):
            for _ in range(2):
                ctx.rexi_linear_step(a, b, w.dt, U0, U1, side)
            side.synchronize()
            # a graph of `reps` stages, so host launch gaps do not count
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=side):
                for _ in range(reps):
                    ctx.rexi_linear_step(a, b, w.dt, U0, U1, side)
            ms = _timed(g.replay, 3, side) / reps
        out[key] = {"N": w.N, "p0": w.p0, "tuning": ctx.get_tuning(), "ms_per_stage": ms,
                    "term_solves_per_s": w.N / (ms * 1e-3),
                    "sim_time_per_wall_rexi_stage": w.dt / (ms * 1e-3), **_field_errors(U1.cpu().numpy(), ref)}
        ctx.close()
    out["fp64_speedup_at_equal_error"] = out["fp32"]["ms_per_stage"] / out["fp64"]["ms_per_stage"]
    return out


def schemes_arm(reps):
    """Time per step of the time-stepping schemes built on the same kernels, T255
    on 768 x 384, dt = 3600 s, N = 800 (FP64 solves and transforms): the
    Strang-split REXI step (L = L_g + L_c), the fast variant with REXI on L_g
    only, Crank-Nicolson in place of REXI, and ETD2RK."""
    import torch

    from paper_1805_06557_amd import api, configs
    from paper_1805_06557_amd.inputs import jet_state

    w = configs.T255_FP64
    a, b0, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    _, b1, _, _ = api.rexi_coefficients(api.FN_PSI1, w.N, w.p0, w.y)
    _, b2, _, _ = api.rexi_coefficients(api.FN_PSI2, w.N, w.p0, w.y)
    ctx = api.SWE(w.L, w.nlat, w.nlon, prec=0)
    U = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    V = torch.empty_like(U)
    stream = torch.cuda.current_stream()
    runs = {
        "l_rexi_n_erk_ver1": lambda: ctx.split_step(api.SPLIT_REXI_V1, a, b0, w.dt, U, V, stream),
        "lg_rexi_lc_n_erk_ver1": lambda: ctx.split_step(api.SPLIT_LG_REXI_V1, a, b0, w.dt, U, V, stream),
        "l_irk_n_erk_ver1 (Crank-Nicolson)": lambda: ctx.split_step(api.SPLIT_CN_V1, None, None, w.dt, U, V, stream),
        "l_rexi_n_etdrk": lambda: ctx.etdrk2_step(a, b0, b1, b2, w.dt, U, V, stream),
    }
    out = {"workload": "T255 on 768x384, dt=3600 s, N=800 (p0=12), FP64"}
    for name, fn in runs.items():
        fn()
        ms = _timed(fn, reps, stream)
        out[name] = {"ms_per_step": ms, "sim_time_per_wall": w.dt / (ms * 1e-3)}
    ctx.close()
    return out


def graph_steps(ctx, full, alpha, beta, w, U, V, steps):
    """The same steps replayed from one captured HIP graph of two steps
    (U -> V -> U): three replays, each from the same state with eager work in
    between, must equal two eager steps bit for bit; then the replays are timed."""
    import torch

    def two(s):
        # U -> U over two steps (a full step as one two-step swe_strang_steps call)
        if full:
            ctx.strang_steps(alpha, beta, w.dt, 2, U, U, s)
        else:
            ctx.rexi_linear_step(alpha, beta, w.dt, U, V, s)
            ctx.rexi_linear_step(alpha, beta, w.dt, V, U, s)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    ctx.profile(False)
    with torch.cuda.stream(side):
        S0 = U.clone()
        two(side)
        ref = U.clone()
        g = torch.cuda.CUDAGraph()
        U.copy_(S0)
        with torch.cuda.graph(g, stream=side):
            two(side)
        same = True
        for _ in range(3):
            U.copy_(S0)
            side.synchronize()
            g.replay()
            side.synchronize()
            same = same and bool(torch.equal(U, ref))
            V.zero_()
        reps = max(1, steps // 2)
        ms = _timed(g.replay, reps, side) / 2.0
    torch.cuda.synchronize()
    return {"ms_per_step": ms, "term_solves_per_s": w.N / (ms * 1e-3), "sim_time_per_wall": w.dt / (ms * 1e-3),
            "replays_bit_identical_to_eager": same,
            "note": "two steps per graph; eager launches of the same kernels are the headline value"}


def ensemble_arm(reps):
    """64 linear-SWE members of mixed truncation and pole count (FP32 solves):
    one fused ensemble launch (eager and replayed from a captured graph) against
    one rexi_linear_step per member."""
    import torch

    from paper_1805_06557_amd import api, configs
    from paper_1805_06557_amd.inputs import random_state

    plan = configs.ensemble_plan()
    members = []
    for m in plan:
        ctx = api.SWE(m["L"], prec=1)
        a, b, _, _ = api.rexi_coefficients(api.FN_EXP, m["N"], m["p0"], m["y"])
        U0 = torch.from_numpy(random_state(m["L"], m["seed"])).cuda()
        members.append((ctx, a, b, m["dt"], U0, torch.empty_like(U0)))
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        api.rexi_linear_step_batched(members, stream=stream)
        stream.synchronize()
        fused = [m[5].clone() for m in members]
        eager = _timed(lambda: api.rexi_linear_step_batched(members, stream=stream), reps, stream)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            api.rexi_linear_step_batched(members, stream=stream)
        graph = _timed(g.replay, reps, stream)

        def separate():
            for ctx, a, b, dt, U0, U1 in members:
                ctx.rexi_linear_step(a, b, dt, U0, U1, stream)
        separate()
        stream.synchronize()
        same = all(bool(torch.equal(f, m[5])) for f, m in zip(fused, members))
        sep = _timed(separate, reps, stream)
    total_n = sum(m["N"] for m in plan)
    for m in members:
        m[0].close()
    return {"members": len(plan), "truncations": sorted({m["L"] for m in plan}), "total_poles": total_n,
            "ms_fused_eager": eager, "ms_fused_graph": graph, "ms_one_launch_per_member": sep,
            "every_member_bit_identical_to_its_single_call": same,
            "term_solves_per_s_graph": total_n / (graph * 1e-3)}


def stream_arm(w, reps):
    """The factor-streaming schedule of the REXI solve (pivots cached per contour
    and dt, read by both sweeps) on this workload's REXI problem, FP32 and FP64
    solves: HIP events around every solve launch; algorithmic bytes 16 B (FP32)
    or 32 B (FP64) per pole-unknown against the 8 TB/s HBM peak, with the
    counter-measured traffic where the profiles hold it for this kernel source."""
    import torch

    from paper_1805_06557_amd import api
    from paper_1805_06557_amd.inputs import jet_state

    a, b, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    U0 = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    U1 = torch.empty_like(U0)
    stream = torch.cuda.current_stream()
    out = {}
    for key, prec in (("fp32", api.PREC_FP32_SOLVE), ("fp64", 0)):
        ctx = api.SWE(w.L, prec=prec)
        ctx.set_tuning(solver=api.SOLVER_STREAM)
        ctx.rexi_linear_step(a, b, w.dt, U0, U1, stream)            # builds the cached pivots
        ctx.sync()
        ctx.profile_kernels([api.KERNEL_SOLVE])
        for _ in range(reps):
            ctx.rexi_linear_step(a, b, w.dt, U0, U1, stream)
        ms, n = ctx.profile_read(api.KERNEL_SOLVE)
        ctx.sync()
        tuning = ctx.get_tuning()
        ctx.close()
        per = ms / max(n, 1)
        nbytes = STREAM_BYTES_PER_POLE_UNKNOWN[key == "fp32"] * pole_unknowns(w.L, w.N)
        gbs = nbytes / (per * 1e-3) / 1e9
        out[key] = {"bound": "hbm", "kernel": "rexi_chain_kernel (streaming schedule)", "achieved": gbs,
                    "peak": PEAK_HBM, "unit": "GB/s", "frac": gbs / PEAK_HBM,
                    "traffic": measured_traffic(f"{w.name}-stream-{key}", tuning),
                    "algorithmic_bytes_per_launch": nbytes, "avg_kernel_ms": per, "launches": n,
                    "tuning": tuning}
    return out


def split_mfma_flops_batch(L, nlat, nf):
    """Matrix-core flops of one scalar-field split Legendre launch over nf fields
    (8 fields = 16 real columns per 16-column product; three bf16 products per
    16x16x16 tile and K step, padding rows and latitudes included)."""
    hpad, rows = _split_blocks(L, nlat)
    groups = (nf + 7) // 8
    return groups * 3 * (hpad // 16) * (rows // 16) * 2 * 16 * 16 * 16


def legendre_batch_arm(reps, nf=64):
    """The Legendre stage of the transforms of many fields on one grid (T255 on
    768 x 384, nf scalar fields): synthesis and analysis with the split-BF16
    matrix-core kernels and with the FP64 kernels, HIP events around the
    Legendre launches only.  Reports the matrix-core rate against the 2.5 PFLOP/s
    dense bf16 peak and the algorithmic bytes (table once per 8-field group,
    spectra in or out, Fourier coefficients out or in, complex128)."""
    import numpy as np
    import torch

    from paper_1805_06557_amd import api
    from paper_1805_06557_amd.inputs import random_field

    L, nlat, nlon = 255, 384, 768
    rng = np.random.default_rng(77)
    spec = torch.from_numpy(np.stack([random_field(L, rng, 1.0) for _ in range(nf)])).cuda()
    grid = torch.empty((nf, nlat, nlon), dtype=torch.float64, device="cuda")
    back = torch.empty_like(spec)
    stream = torch.cuda.current_stream()
    out = {"workload": f"T{L} on {nlon}x{nlat}, {nf} scalar fields per call"}
    four_bytes = nf * (L + 1) * nlat * 16
    spec_bytes = nf * n_modes(L) * 16
    for key, prec in (("bf16_split", api.PREC_BF16_SPLIT), ("fp64", 0)):
        ctx = api.SWE(L, nlat, nlon, prec=prec)
        ctx.sh_synthesis(spec, grid, nf, stream)
        ctx.sh_analysis(grid, back, nf, stream)
        ctx.sync()
        ctx.profile_kernels([api.KERNEL_LEG_SYNTH, api.KERNEL_LEG_ANAL])
        for _ in range(reps):
            ctx.sh_synthesis(spec, grid, nf, stream)
            ctx.sh_analysis(grid, back, nf, stream)
        ms_s, n_s = ctx.profile_read(api.KERNEL_LEG_SYNTH)
        ms_a, n_a = ctx.profile_read(api.KERNEL_LEG_ANAL)
        ctx.sync()
        ctx.close()
        syn, ana = ms_s / max(n_s, 1), ms_a / max(n_a, 1)
        entry = {"synth_ms": syn, "anal_ms": ana}
        if prec:
            fl = split_mfma_flops_batch(L, nlat, nf)
            tb = split_table_bytes(L, nlat) * ((nf + 7) // 8)
            entry.update({
                "mfma_flops_per_launch": fl, "peak_TFLOP_s": PEAK_BF16_MFMA,
                "synth_TFLOP_s": fl / (syn * 1e-3) / 1e12, "anal_TFLOP_s": fl / (ana * 1e-3) / 1e12,
                "synth_frac": fl / (syn * 1e-3) / 1e12 / PEAK_BF16_MFMA,
                "anal_frac": fl / (ana * 1e-3) / 1e12 / PEAK_BF16_MFMA,
                "table_bytes_per_launch": tb,
            })
        else:
            tb = 0
        io = four_bytes + spec_bytes
        entry.update({"algorithmic_bytes_per_launch": io + tb, "fourier_and_spectral_bytes": io,
                      "synth_GB_s": (io + tb) / (syn * 1e-3) / 1e9, "anal_GB_s": (io + tb) / (ana * 1e-3) / 1e9})
        out[key] = entry
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="T255-fp32-bf16")
    ap.add_argument("--stage", choices=["auto", "rexi"], default="auto")
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--solver", choices=["default", "fused", "stream", "hybrid"], default="default",
                    help="REXI chain-solve schedule")
    ap.add_argument("--seg-rows", type=int, default=0, help="REXI solve segment length (8, 16, 32; 0 = default)")
    ap.add_argument("--waves", type=int, default=0, help="REXI solve waves per workgroup (1, 2, 4; 0 = default)")
    ap.add_argument("--ppl", type=int, default=0, help="REXI solve poles per lane (1, 2; 0 = default)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run 5 device-to-device copies of BYTES (reference kernel for HBM counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the REXI solve of the main workload (default: the library's launch shape)")
    ap.add_argument("--no-arms", action="store_true",
                    help="skip the FP32-vs-FP64 equal-error arm and the ensemble arm")
    ap.add_argument("--only-legendre-batch", action="store_true",
                    help="only run the batched Legendre arm (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; multi-GPU sharding is designed but not built "
              "(see the design notes).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        src = torch.ones(args.copy_calibration // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 4, "copies": 5}))
        return

    from paper_1805_06557_amd import api, configs
    from paper_1805_06557_amd.inputs import jet_state

    if args.only_legendre_batch:
        print(json.dumps({"legendre_batched": legendre_batch_arm(max(3, args.steps // 4))}))
        return
    w = configs.ALL[args.workload]
    alpha, beta, _, _ = api.rexi_coefficients(api.FN_EXP, w.N, w.p0, w.y)
    full = args.stage == "auto" and w.nlat > 0
    limit = w.extra.get("max_steps") if full else None
    if limit:
        # the jet state of this workload grows unstable under the explicit stage
        # after a few steps: one warm-up and `limit` timed steps
        args.warmup = min(args.warmup, 1)
        args.steps = min(args.steps, limit)
    ctx = api.SWE(w.L, w.nlat if full else 0, w.nlon if full else 0, prec=w.prec)
    solver = {"default": 0, "fused": api.SOLVER_FUSED, "stream": api.SOLVER_STREAM,
              "hybrid": api.SOLVER_HYBRID}[args.solver]
    if solver or args.seg_rows or args.waves or args.ppl:
        ctx.set_tuning(solver=solver, seg_rows=args.seg_rows, waves=args.waves, poles_per_lane=args.ppl)
    U = torch.from_numpy(jet_state(w.L, w.seed)).cuda()
    V = torch.empty_like(U)
    stream = torch.cuda.current_stream()
    if args.autotune and not (solver or args.seg_rows or args.waves or args.ppl):
        # pick the REXI solve's schedule and launch shape on this problem (outside the timed region)
        ctx.autotune(alpha, beta, w.dt, U, V, reps=3, stream=stream)

    def step(src, dst):
        if full:
            ctx.strang_step(alpha, beta, w.dt, src, dst, stream)
        else:
            ctx.rexi_linear_step(alpha, beta, w.dt, src, dst, stream)

    def run_steps(n, src, dst):
        """n steps from src; returns (result, other buffer).  A full step runs as
        one swe_strang_steps call (bit-identical to n single steps; in split
        precision it fuses the last analysis of a step with the next synthesis)."""
        if full:
            ctx.strang_steps(alpha, beta, w.dt, n, src, dst, stream)
            return dst, src
        for _ in range(n):
            step(src, dst)
            src, dst = dst, src
        return src, dst

    ctx.profile(True)
    if args.warmup:
        U, V = run_steps(args.warmup, U, V)
    torch.cuda.synchronize()
    # the factorization of the streaming schedules is built by the first call
    fact_ms, fact_n = ctx.profile_read(api.KERNEL_FACTOR)
    for kid in range(api.KERNEL_FACTOR):
        ctx.profile_read(kid)
    ctx.profile_read(api.KERNEL_LEG_FUSED)
    # timed region: HIP events around the dominant kernel's launches only
    ctx.profile_kernels([api.KERNEL_SOLVE])
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    U, V = run_steps(args.steps, U, V)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(stop)
    solve_ms_timed, solve_n_timed = ctx.profile_read(api.KERNEL_SOLVE)
    # a second pass of the same steps with HIP events around every kernel launch
    # for the per-stage breakdown (their gaps would add to a timed step)
    ctx.profile(True)
    U, V = run_steps(args.steps, U, V)
    torch.cuda.synchronize()
    stage_ms = {}
    split = bool(w.prec & (api.PREC_BF16_SPLIT | api.PREC_FP16_SPLIT))
    # in a split-precision Strang step the pole sum is fused with the synthesis of its result
    reduce_name = "pole_sum_synth_kernel" if (full and split) else "sum_partials_kernel"
    for kid, name in [(api.KERNEL_SOLVE, "rexi_chain_kernel"), (api.KERNEL_REDUCE, reduce_name),
                      (api.KERNEL_LEG_SYNTH, "legendre_synth_kernel"), (api.KERNEL_RING, "ring_kernel"),
                      (api.KERNEL_LEG_ANAL, "legendre_anal_kernel"),
                      (api.KERNEL_LEG_FUSED, "legendre_anal_synth_kernel")]:
        ms, n = ctx.profile_read(kid)
        stage_ms[name] = {"ms_per_step": ms / args.steps, "launches_per_step": n / args.steps,
                          "ms_per_launch": ms / max(n, 1)}
    solve_ms, solve_n = solve_ms_timed, solve_n_timed
    ctx.profile(False)
    try:
        ctx.sync()                     # the library's device-side status: non-finite outputs
    except api.RexiError as e:
        print(f"bench.py: {e}", file=sys.stderr)
        sys.exit(3)

    ms_per_step = ms_total / args.steps
    fp32 = bool(w.prec & api.PREC_FP32_SOLVE)
    peak = PEAK_FP32_VALU if fp32 else PEAK_FP64_VALU
    tuning = ctx.get_tuning()
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
                        + ((", split-BF16 Legendre + FP64 FFTs" if w.prec & api.PREC_BF16_SPLIT else
                            ", split-FP16 Legendre + FP64 FFTs" if w.prec & api.PREC_FP16_SPLIT else
                            ", FP64 transforms") if full else ""),
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
            "traffic": measured_traffic(w.name, tuning),
            "avg_kernel_ms": avg_solve_ms,
            "launches": solve_n,
            "algorithmic_flops_per_launch": solve_flops(w.L, w.N),
            "flops_per_pole_unknown": FLOPS_PER_POLE_UNKNOWN,
            "pole_unknowns_per_launch": pole_unknowns(w.L, w.N),
            "peak_note": "vector ALU peak without packed FP32: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz",
            "frac_of_published_fp32_peak": achieved / PEAK_FP32_PACKED if fp32 else None,
            "published_fp32_peak": PEAK_FP32_PACKED if fp32 else None,
            "tuning": tuning,
        },
        "kernels": stage_ms,
        "setup": {"rexi_factor_kernel_ms": fact_ms / max(fact_n, 1), "launches": fact_n},
    }
    oracle_ref = None
    if not args.no_cpu_baseline:
        u0 = jet_state(w.L, w.seed)
        oracle_ref, out["cpu_baseline"] = oracle_step(w, u0, full, args.cpu_seconds)
        if oracle_ref is not None:
            out["step_error_vs_oracle"] = step_error_vs_oracle(ctx, w, alpha, beta, u0, oracle_ref, full)
    if full and (w.prec & (api.PREC_BF16_SPLIT | api.PREC_FP16_SPLIT)):
        syn = stage_ms["legendre_synth_kernel"]["ms_per_launch"]
        ana = stage_ms["legendre_anal_kernel"]["ms_per_launch"]
        fus = stage_ms["legendre_anal_synth_kernel"]
        fl = split_mfma_flops(w.L, w.nlat)
        out["legendre_mfma"] = {
            "precision": ("bf16" if w.prec & api.PREC_BF16_SPLIT else "fp16") + " hi/lo split, 3 products, FP32 accumulation",
            "mfma_flops_per_launch": fl,
            "synth_TFLOP_s": fl / (syn * 1e-3) / 1e12, "anal_TFLOP_s": fl / (ana * 1e-3) / 1e12,
            "peak_TFLOP_s": PEAK_BF16_MFMA,
            "synth_frac": fl / (syn * 1e-3) / 1e12 / PEAK_BF16_MFMA,
            "anal_frac": fl / (ana * 1e-3) / 1e12 / PEAK_BF16_MFMA,
            "table_bytes_per_launch": split_table_bytes(w.L, w.nlat),
            "synth_GB_s": split_table_bytes(w.L, w.nlat) / (syn * 1e-3) / 1e9,
            "anal_GB_s": split_table_bytes(w.L, w.nlat) / (ana * 1e-3) / 1e9,
        }
        if fus["launches_per_step"] > 0:
            # a Heun step's first analysis fused with the next synthesis: both
            # contractions and both tables per launch
            t = fus["ms_per_launch"] * 1e-3
            out["legendre_mfma"].update({
                "fused_anal_synth_launches_per_step": fus["launches_per_step"],
                "fused_TFLOP_s": 2 * fl / t / 1e12,
                "fused_frac": 2 * fl / t / 1e12 / PEAK_BF16_MFMA,
                "fused_GB_s": 2 * split_table_bytes(w.L, w.nlat) / t / 1e9,
            })
    out["graph"] = graph_steps(ctx, full, alpha, beta, w, U, V, args.steps)
    ctx.close()
    if not args.no_arms:
        out["roofline_stream"] = stream_arm(w, max(3, args.steps // 2))
        out["legendre_batched"] = legendre_batch_arm(max(3, args.steps // 4))
        out["fp32_vs_fp64_at_equal_error"] = equal_error_arm(max(3, args.steps // 2),
                                                             with_oracle=not args.no_cpu_baseline)
        out["ensemble"] = ensemble_arm(max(3, args.steps // 2))
        out["schemes"] = schemes_arm(max(3, args.steps // 4))
    # the cpu_baseline dict goes last in the line
    if "cpu_baseline" in out:
        out["cpu_baseline"] = out.pop("cpu_baseline")
    print(json.dumps(out))


if __name__ == "__main__":
    main()

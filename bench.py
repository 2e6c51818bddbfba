#!/usr/bin/env python3
"""Benchmark of the fused Poisson relaxation on one MI355X.

A step is one pass of the whole hot path over one synthetic batch: 200 fused
damped-Jacobi sweeps (omega = 2/3) of the 4096 x 4096 FP64 cell-centred
Poisson problem, f ~ Uniform[-1,1] (PCG64 seed 2), phi0 = 0, homogeneous
Dirichlet boundary, ending with the max-norm and sum of squares of the final
residual -- stencil, residual, update and temporal blocking all inside the
HIP kernels.  value = cell-updates per second (n^2 * 200 / step time).

Prints one JSON line.  Extra keys: `roofline` of the dominant kernel (the
fused relaxation kernel), `cpu_baseline` (the CPU oracle on a bounded sample
of the same workload), and `variants` (FP64/FP32 at 1-8 sweeps per launch, the
unfused three-kernel sweep, the standalone stencil).

  python bench.py [--steps K] [--warmup W] [--tblock T] [--no-variants] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N = 4096
SWEEPS = 200
OMEGA = 2.0 / 3.0
BYTES_PER_CELL = {"f64": 24, "f32": 12, "bf16": 6}  # read phi + f, write phi', per launch
# FP64 operations per cell per sweep: stencil 4 adds + 1 multiply, update 2 multiplies +
# 2 adds.  Bit-exactness forbids fused multiply-add, so the attainable FP64 vector rate
# is one add or multiply per lane per clock: 256 CUs x 64 lanes x 2.4 GHz = 39.3 TFLOP/s
# (the 78.6 TFLOP/s figure counts an FMA as two).
FLOPS_PER_CELL_SWEEP = 9
FP64_NOFMA_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
METRIC = ("Gcell-updates/s & %HBM peak (fused relax); time-to-1e-10 residual learned/mixed vs plain")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def setup(n, dt_name):
    import torch
    import paper_2307_07931_amd as px
    import workloads as W
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt_name]
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    f_host = W.uniform_rhs(n, W.SEED_UNIFORM_4096)
    phi0 = px.alloc_grid(n, tdt)
    phi_out = px.alloc_grid(n, tdt)
    f = px.alloc_rhs(n, tdt)
    f[:, :n] = torch.from_numpy(f_host).cuda().to(torch.float32 if dt_name != "f64" else torch.float64).to(tdt)
    return dict(n=n, h=h, lam=lam, phi0=phi0, phi_out=phi_out, f=f, tdt=tdt, f_host=f_host)


def time_region(fn, reps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3  # seconds


def relax_fn(px, d, ctx, norms, tblock, sweeps=SWEEPS, resmode=None):
    rm = px.RES_FINAL if resmode is None else resmode
    return lambda: px.relax_fused(d["phi0"], d["phi_out"], d["n"], d["f"], d["h"], d["lam"], sweeps,
                                  ctx, tblock=tblock, resmode=rm, norms=norms)


def variants(px, ctx, norms):
    import torch
    out = {}
    for dt in ("f64", "f32"):
        d = setup(N, dt)
        ctx.reserve(N, d["phi0"].stride(0), px.dtype_code(d["phi0"]))
        for tb in range(1, 9):
            reps = 3
            t = time_region(relax_fn(px, d, ctx, norms, tb), reps=reps, warmup=2)
            launches = -(-SWEEPS // tb)
            gcell = N * N * SWEEPS * reps / t / 1e9
            gbs = BYTES_PER_CELL[dt] * N * N * launches * reps / t / 1e9
            out[f"fused_{dt}_k{tb}"] = {"gcell_s": round(gcell, 2), "alg_GBs": round(gbs, 1),
                                        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
            log(f"  fused {dt} k={tb}: {gcell:8.1f} Gcell/s  {gbs:7.1f} GB/s algorithmic")
        tmp = torch.zeros((N, N), dtype=d["tdt"], device="cuda")
        es = 8 if dt == "f64" else 4

        def unfused():
            for _ in range(SWEEPS):
                px.apply_stencil(d["phi0"], N, tmp)
                px.jacobi_update(d["phi0"], N, tmp, d["f"], d["h"], d["lam"])
                px.residual(d["phi0"], N, d["f"], d["h"], norms, ctx)

        t = time_region(unfused, reps=1, warmup=0)
        d["phi0"].zero_()
        out[f"unfused_{dt}"] = {"gcell_s": round(N * N * SWEEPS / t / 1e9, 2),
                                "alg_GBs": round(8 * es * N * N * SWEEPS / t / 1e9, 1)}
        log(f"  unfused {dt} (stencil -> temp, update, residual): {N * N * SWEEPS / t / 1e9:8.1f} Gcell/s")
        t = time_region(lambda: px.apply_stencil(d["phi0"], N, tmp), reps=50, warmup=5)
        out[f"apply_stencil_{dt}"] = {"gcell_s": round(N * N * 50 / t / 1e9, 2),
                                      "alg_GBs": round(2 * es * N * N * 50 / t / 1e9, 1)}
        log(f"  apply_stencil {dt}: {2 * es * N * N * 50 / t / 1e9:8.1f} GB/s algorithmic")
        del d, tmp
        torch.cuda.empty_cache()
    return out


def cpu_baseline(sample_sweeps):
    import numpy as np
    import oracle
    import workloads as W
    oracle.build()
    n = N
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    f = W.uniform_rhs(n, W.SEED_UNIFORM_4096)
    phi0 = np.zeros((n + 2, n + 2))
    t0 = time.perf_counter()
    oracle.relax(phi0, f, n, h, lam, sample_sweeps)
    t = time.perf_counter() - t0
    return {"value": round(n * n * sample_sweeps / t / 1e9, 5), "unit": "Gcell-updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n}x{n} FP64, same f and phi0, {sample_sweeps} sweeps + final residual "
                      f"(of the {SWEEPS}), plain three-pass oracle, single thread, {t:.1f} s"}


def mixed_workload(px, ctx):
    """Mixed-precision refinement (FP32 / BF16 inner sweeps, FP64 outer residual and
    update) against plain FP64 relaxation, on |k|^-2 Gaussian-random-field right-hand
    sides.  (a) measured time to max|r| <= 1e-10 max|f| at 256^2 and 512^2, with the
    error of each result against the exact discrete solution (DST); (b) cost per sweep
    at 8192^2 and the time to the FP64-attainable tolerance extrapolated from it and the
    closed-form asymptotic rate of the slowest mode."""
    import math
    import numpy as np
    import torch
    import workloads as W
    from oracle import exact  # CPU reference for the error of each result
    out = {"solves": [], "per_sweep_8192": {}}
    for n in (256, 512):
        f_host = W.grf_rhs(n, W.SEED_GRF_8192)
        ex = exact.dst_solve(f_host, 1.0 / n)
        h = 1.0 / n
        lam = OMEGA * h * h / 4.0
        for mode, name, inner in ((px.SOLVE_PLAIN, "plain_f64", 0), (px.SOLVE_MIXED_F32, "mixed_f32", 64),
                                  (px.SOLVE_MIXED_BF16, "mixed_bf16", 32)):
            phi = px.alloc_grid(n, torch.float64)
            f = px.alloc_rhs(n, torch.float64)
            f[:, :n] = torch.from_numpy(f_host).cuda()
            st = px.solve(phi, n, f, h, lam, ctx, mode=mode, rtol=1e-10, check_every=2048,
                          inner_sweeps=inner, raise_on_error=False)
            err = float(np.abs(phi[1:n + 1, 1:n + 1].cpu().numpy() - ex).max() / np.abs(ex).max())
            rec = {"n": n, "mode": name, "status": st.status, "sweeps": st.sweeps, "seconds": round(st.seconds, 3),
                   "rel_res_max": st.rel_res_max, "rel_err_vs_exact": err}
            out["solves"].append(rec)
            log(f"  mixed/{n}: {rec}")
    # (b) 8192^2: time per sweep of each form
    n = 8192
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    f_host = W.grf_rhs(n, W.SEED_GRF_8192)
    per = {}
    for dt, tdt in (("f64", torch.float64), ("f32", torch.float32), ("bf16", torch.bfloat16)):
        a = px.alloc_grid(n, tdt)
        b = px.alloc_grid(n, tdt)
        f = px.alloc_rhs(n, tdt)
        src = torch.from_numpy(f_host).cuda()
        f[:, :n] = src if dt == "f64" else src.float().to(tdt)
        k, rows, _ = px.autotune(a, b, n, f, ctx)
        t = time_region(lambda: px.relax_fused(a, b, n, f, h, lam, 64, ctx, tblock=0, resmode=px.RES_NONE),
                        reps=5, warmup=2)
        per[dt] = {"s_per_sweep": t / (5 * 64), "k": k, "rows": rows,
                   "gcell_s": round(n * n * 64 * 5 / t / 1e9, 1)}
        del a, b, f, src
        torch.cuda.empty_cache()
    # refinement step (FP64 residual + update + rounding of r) at 8192^2: one mixed solve
    # with a budget of one outer step, timed on the host
    phi = px.alloc_grid(n, torch.float64)
    f = px.alloc_rhs(n, torch.float64)
    f[:, :n] = torch.from_numpy(f_host).cuda()
    for inner, mode in ((64, px.SOLVE_MIXED_F32), (32, px.SOLVE_MIXED_BF16)):
        phi.zero_()
        st = px.solve(phi, n, f, h, lam, ctx, mode=mode, rtol=0.0, max_sweeps=inner * 4, inner_sweeps=inner,
                      raise_on_error=False)
        per["mixed_" + ("f32" if mode == px.SOLVE_MIXED_F32 else "bf16")] = {
            "s_per_sweep_incl_refine": st.seconds / st.sweeps, "inner": inner, "outer_steps": st.outer_steps}
    g = exact.mode_factor(n, 1, 1, OMEGA)
    floor = 5.6e-10  # FP64 attainable relative residual for this field at 8192^2 (exact solution rounded)
    tau = max(1e-10, 4 * floor)
    sweeps = math.log(tau) / math.log(g)
    t_plain = sweeps * per["f64"]["s_per_sweep"]
    for key in ("mixed_f32", "mixed_bf16"):
        per[key]["extrapolated_seconds_to_tau"] = sweeps * per[key]["s_per_sweep_incl_refine"]
        per[key]["speedup_vs_plain_f64"] = t_plain / per[key]["extrapolated_seconds_to_tau"]
    per["plain_f64_extrapolated_seconds_to_tau"] = t_plain
    per["tau_eff"] = tau
    per["sweeps_to_tau_closed_form"] = sweeps
    out["per_sweep_8192"] = per
    log(f"  mixed/8192: {per}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--tblock", type=int, default=0,
                    help="sweeps per launch; 0 = autotuned (k, tile rows) before timing")
    ap.add_argument("--rows", type=int, default=0, help="tile rows (with --tblock; 0 = default)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy 5 times (the known-size kernel "
                         "that scales the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--workload", choices=["relax", "mixed"], default="relax",
                    help="relax: the fused relaxation benchmark (default); mixed: mixed-precision "
                         "refinement against plain FP64 (time to tolerance)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=24)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the relaxation is sharded "
              f"by box decomposition only in design, not in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2307_07931_amd as px
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "copy", "bytes_read": a.numel() * 8,
                          "bytes_written": b.numel() * 8, "dispatches": 5}), flush=True)
        return
    px.lib()
    torch.cuda.set_device(0)
    ctx = px.Context(0)
    norms = torch.zeros(2, dtype=torch.float64, device="cuda")
    if args.workload == "mixed":
        t0 = time.perf_counter()
        res = mixed_workload(px, ctx)
        p8 = res["per_sweep_8192"]
        print(json.dumps({"metric": METRIC, "workload": "mixed_precision_refinement_grf",
                          "value": round(p8["mixed_f32"]["speedup_vs_plain_f64"], 3),
                          "unit": "x time-to-tolerance speedup (mixed FP32 vs plain FP64, 8192^2, extrapolated)",
                          "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "results": res,
                          "wall_s": round(time.perf_counter() - t0, 1)}), flush=True)
        ctx.close()
        return

    d = setup(N, "f64")
    ctx.reserve(N, d["phi0"].stride(0), px.F64)
    tb = args.tblock
    rows = None
    if args.rows:
        ctx.set_tile_rows(args.rows)
        rows = args.rows
    if tb == 0:
        tb, rows, g = px.autotune(d["phi0"], d["phi_out"], N, d["f"], ctx)
        log(f"autotuned: {tb} sweeps per launch, {rows} rows per tile ({g:.1f} Gcell/s in the tuner)")
    step = relax_fn(px, d, ctx, norms, tb)
    log(f"timing {args.steps} steps of {SWEEPS} sweeps, {N}^2 FP64, {tb} sweeps per launch")
    t = time_region(step, reps=args.steps, warmup=args.warmup)
    ms = t / args.steps * 1e3
    value = N * N * SWEEPS * args.steps / t / 1e9
    launches = -(-SWEEPS // tb)
    # every launch of a step moves 24 B per cell; the step also holds one tiny norm reduction
    per_launch_s = t / (args.steps * launches)
    achieved = BYTES_PER_CELL["f64"] * N * N / per_launch_s / 1e9
    log(f"step {ms:.3f} ms -> {value:.1f} Gcell-updates/s; relax launch {per_launch_s * 1e6:.1f} us "
        f"-> {achieved:.1f} GB/s algorithmic ({achieved / HBM_PEAK_GBS:.1%} of 8 TB/s)")
    res_max = float(norms[0])
    hbm_view = {"achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": BYTES_PER_CELL["f64"] * N * N}
    if tb == 1:
        roofline = {"bound": "hbm", **hbm_view, "traffic": None}
    else:
        # several sweeps per launch: HBM bytes per cell-update fall to 24/k and the
        # kernel is bound by vector ALU issue
        tflops = FLOPS_PER_CELL_SWEEP * N * N * tb / per_launch_s / 1e12
        roofline = {"bound": "alu", "achieved": round(tflops, 3), "peak": round(FP64_NOFMA_PEAK_TFLOPS, 1),
                    "unit": "TFLOP/s", "frac": round(tflops / FP64_NOFMA_PEAK_TFLOPS, 4), "traffic": None,
                    "alg_flops_per_launch": FLOPS_PER_CELL_SWEEP * N * N * tb, "hbm_view": hbm_view}
    roofline["kernel"] = f"relax_tb_kernel<double,2,{tb},*> ({rows or 'default'} rows per tile)"

    var = None if args.no_variants else variants(px, ctx, norms)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_sweeps)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson2d_fused_jacobi_4096sq_fp64_200sweeps", "n": N,
                   "sweeps_per_step": SWEEPS, "sweeps_per_launch": tb, "tile_rows": rows,
                   "omega": OMEGA,
                   "rhs": "uniform[-1,1] PCG64 seed 2", "phi0": 0, "bc": "dirichlet0_cell_centred",
                   "residual": "final max-norm and sum of squares"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "final_res_max": res_max,
        "variants": var,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

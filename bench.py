#!/usr/bin/env python3
"""Benchmark of the fused Poisson relaxation on one MI355X.

A step is one pass of the whole hot path over one synthetic batch: 200 fused
damped-Jacobi sweeps (omega = 2/3) of the 4096 x 4096 FP64 cell-centred
Poisson problem, f ~ Uniform[-1,1] (PCG64 seed 2), phi0 = 0, homogeneous
Dirichlet boundary, ending with the max-norm and sum of squares of the final
residual -- stencil, residual, update and temporal blocking all inside the
HIP kernels.  value = cell-updates per second (n^2 * 200 / step time).

Prints one JSON line.  Extra keys: `roofline` of the dominant kernel (the
fused relaxation kernel), `cpu_baseline` (the CPU oracle on the same workload,
at all host cores and at one thread), `variants` (FP64/FP32 at 1-8 sweeps per
launch, the unfused three-kernel sweep, the standalone stencil) and
`time_to_tolerance` (the metric's second half: measured time to a 1e-10
relative residual at 512^2 of plain FP64, mixed FP32/BF16 refinement and the
refinement loop without and with the network trained in the run, plus the
labelled 8192^2 mixed-precision extrapolation).

  python bench.py [--steps K] [--warmup W] [--tblock T] [--no-variants] [--no-cpu] [--no-ttt]
  python bench.py --workload mixed|learned|batched|net
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
# (the 78.6 TFLOP/s figure counts an FMA as two).  These 9 are the method's count; the
# interior loop forms lambda f once per row and reuses it at every level, so it issues
# 8 per cell-update plus 1 per cell and launch.
FLOPS_PER_CELL_SWEEP = 9
FP64_NOFMA_PEAK_TFLOPS = 256 * 64 * 2.4e9 / 1e12
# HBM traffic of the FP64 fused relaxation at 4096^2, per launch: rocprofv3 --pmc FETCH_SIZE
# and WRITE_SIZE (KiB per dispatch, averaged over the dispatches of a short bench run with
# the given sweeps per launch and tile rows), scaled by what the same counters read for a
# 1 GiB device-to-device copy (FETCH_SIZE 524302.65 KiB -> x 1048576 / 524302.65,
# WRITE_SIZE 1048576 KiB -> x 1).  Valid only for the kernel sources they were taken on
# (sha256 over TRAFFIC_SOURCES); otherwise the bench reports traffic as null.
TRAFFIC_SOURCES = ("relax_kernel.h", "relax_f64.hip", "relax.hip", "px_internal.h")
TRAFFIC_SHA256 = "7fd6930559948e47f25e77125dcc90d5c654d238abac978d37d49644d564df82"
TRAFFIC_SCALE = (1048576.0 / 524302.65, 1.0)
TRAFFIC_KIB = {  # (sweeps per launch, tile rows): (FETCH_SIZE, WRITE_SIZE) KiB per dispatch
    (8, 29): (165920.44, 131264.06), (8, 38): (160775.76, 131264.06), (8, 44): (157887.19, 131264.06),
    (8, 47): (156024.23, 131264.06), (1, 47): (147381.25, 131264.16),
}
# The same launches' memory-side request counters (TCC_EA0_RDREQ_DRAM_32B_sum and
# TCC_EA0_WRREQ_WRITE_DRAM_32B_sum, 32-byte units, no scaling: the copy reads and writes
# exactly its 1 GiB in them).  They count L2 misses sent to memory; no gfx950 counter
# separates Infinity-Cache hits from HBM accesses.
TRAFFIC_DRAM_32B = {(8, 47): (9838615, 4200450), (1, 47): (9430598, 4200454)}
VARIANT_ROWS = (12, 16, 20, 29, 38, 47, 64, 96)  # tile heights tried for each fixed k in the variants
METRIC = ("Gcell-updates/s & %HBM peak (fused relax); time-to-1e-10 residual learned/mixed vs plain")


def measured_traffic(k, rows):
    """HBM bytes per launch of the FP64 relaxation at 4096^2 from the counter table, or
    None if the kernel sources changed since it was taken or the configuration is absent."""
    import hashlib
    src = b"".join(open(os.path.join(ROOT, "paper_2307_07931_amd", "csrc", f), "rb").read()
                   for f in TRAFFIC_SOURCES)
    if hashlib.sha256(src).hexdigest() != TRAFFIC_SHA256 or (k, rows) not in TRAFFIC_KIB:
        return None
    fk, wk = TRAFFIC_KIB[(k, rows)]
    out = {"read": fk * 1024 * TRAFFIC_SCALE[0], "write": wk * 1024 * TRAFFIC_SCALE[1]}
    if (k, rows) in TRAFFIC_DRAM_32B:
        dr, dw = TRAFFIC_DRAM_32B[(k, rows)]
        out["memory_side"] = {"read": dr * 32, "write": dw * 32}
    return out


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


def elementwise_ceiling(n, reps=10):
    """Bandwidth of torch's own a + b -> c over three FP64 arrays of a grid's size: the
    traffic pattern of one sweep (two arrays in, one out, 24 B per element) with no
    stencil, i.e. what a streaming kernel practically gets out of HBM here."""
    import torch
    a = torch.ones((n + 2) * (n + 2), dtype=torch.float64, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    best = time_region(lambda: torch.add(a, b, out=c), reps=1, warmup=2)
    for _ in range(reps - 1):
        best = min(best, time_region(lambda: torch.add(a, b, out=c), reps=1, warmup=0))
    del a, b, c
    torch.cuda.empty_cache()
    return 24 * (n + 2) * (n + 2) / best / 1e9


def variants(px, ctx, norms):
    import torch
    out = {}
    ceil = elementwise_ceiling(N)
    out["elementwise_ceiling_f64"] = {"GBs": round(ceil, 1), "hbm_frac": round(ceil / HBM_PEAK_GBS, 4),
                                      "kernel": "torch add a + b -> c, three FP64 arrays of 4098^2"}
    log(f"  elementwise ceiling (a + b -> c, FP64): {ceil:7.1f} GB/s")
    for dt in ("f64", "f32"):
        d = setup(N, dt)
        ctx.reserve(N, d["phi0"].stride(0), px.dtype_code(d["phi0"]))
        for tb in range(1, 9):
            # tile height for this k: the fastest of a few (one timed step each)
            best_rows, best_t = 0, float("inf")
            for rows in VARIANT_ROWS:
                ctx.set_tile_rows(rows)
                tr = time_region(relax_fn(px, d, ctx, norms, tb), reps=1, warmup=1)
                if tr < best_t:
                    best_rows, best_t = rows, tr
            ctx.set_tile_rows(best_rows)
            reps = 3
            t = time_region(relax_fn(px, d, ctx, norms, tb), reps=reps, warmup=1)
            ctx.set_tile_rows(0)
            launches = -(-SWEEPS // tb)
            gcell = N * N * SWEEPS * reps / t / 1e9
            gbs = BYTES_PER_CELL[dt] * N * N * launches * reps / t / 1e9
            out[f"fused_{dt}_k{tb}"] = {"gcell_s": round(gcell, 2), "alg_GBs": round(gbs, 1),
                                        "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "tile_rows": best_rows}
            if dt == "f64" and tb == 1:
                out["fused_f64_k1"]["frac_of_elementwise_ceiling"] = round(gbs / ceil, 4)
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


def host_cpu():
    """nproc, the CPUs this process may use, and the model name from lscpu."""
    import subprocess
    info = {"nproc": os.cpu_count()}
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            key, _, val = line.partition(":")
            if key.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core"):
                info[key.strip()] = val.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    return info


def cpu_baseline(sample_sweeps):
    """The oracle (plain three-pass FP64 sweeps, row loops over OpenMP threads) on the same
    4096^2 problem: the full step at every host core it may use, and at one thread."""
    import numpy as np
    import oracle
    import workloads as W
    oracle.build()
    n = N
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    f = W.uniform_rhs(n, W.SEED_UNIFORM_4096)
    phi0 = np.zeros((n + 2, n + 2))
    res = {}
    for threads in (oracle.default_threads(), 1):
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        oracle.relax(phi0, f, n, h, lam, sample_sweeps)
        res[threads] = time.perf_counter() - t0
        log(f"  cpu oracle, {threads} thread(s): {sample_sweeps} sweeps in {res[threads]:.1f} s")
    oracle.set_threads(oracle.default_threads())
    cores = oracle.default_threads()
    rate = {k: round(n * n * sample_sweeps / v / 1e9, 5) for k, v in res.items()}
    return {"value": rate[cores], "unit": "Gcell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n}x{n} FP64, same f and phi0, {sample_sweeps} sweeps + final residual (of the {SWEEPS}), "
                      f"plain three-pass oracle, {cores} OpenMP threads, {res[cores]:.1f} s",
            "single_thread": {"value": rate[1], "cores": 1, "seconds": round(res[1], 2)},
            "host": host_cpu()}


def exact_solution(f):
    """The exact discrete solution of L u = f (5-point Laplacian / h^2, cell-centred,
    homogeneous Dirichlet by odd reflection) by the type-II sine transform, which
    diagonalises L: used to state the error of each result."""
    import numpy as np
    from scipy import fft as sfft
    n = f.shape[0]
    k = np.arange(1, n + 1, dtype=np.float64)
    lam = -4.0 * n * n * np.sin(k * np.pi / (2 * n)) ** 2
    return sfft.idstn(sfft.dstn(f, type=2, norm="ortho") / (lam[:, None] + lam[None, :]), type=2, norm="ortho")


def slowest_mode_factor(n):
    """Per-sweep damping of the smoothest error mode under damped Jacobi (omega = 2/3):
    1 - omega * (sin^2(pi/2n) + sin^2(pi/2n))."""
    import math
    return 1.0 - OMEGA * 2.0 * math.sin(math.pi / (2 * n)) ** 2


def tune_sizes(px, ctx, n, f_host, dtypes=("f64", "f32", "bf16")):
    """Autotunes the relaxation for n^2 grids of each element type (the grids the solvers
    use have the same pitch), so that small, latency-bound grids get short bands."""
    import torch
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
    for dt in dtypes:
        a = px.alloc_grid(n, tdt[dt])
        b = px.alloc_grid(n, tdt[dt])
        f = px.alloc_rhs(n, tdt[dt])
        src = torch.from_numpy(f_host).cuda()
        f[:, :n] = src if dt == "f64" else src.float().to(tdt[dt])
        k, rows, g = px.autotune(a, b, n, f, ctx)
        log(f"  tuned {n}^2 {dt}: k={k} rows={rows} ({g:.1f} Gcell/s)")


DEFAULT_INNER_SWEEPS = {"mixed_f32": 1024, "mixed_bf16": 128}  # the library's defaults


def mixed_solves(px, ctx, n, seed):
    """Measured time to max|r| <= 1e-10 max|f| at n^2 (|k|^-2 GRF f) of plain FP64
    relaxation and FP64 refinement around FP32 / BF16 inner sweeps, with the error of each
    result against the exact discrete solution (DST)."""
    import numpy as np
    import torch
    import workloads as W
    f_host = W.grf_rhs(n, seed)
    ex = exact_solution(f_host)
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    tune_sizes(px, ctx, n, f_host)
    recs = []
    for mode, name in ((px.SOLVE_PLAIN, "plain_f64"), (px.SOLVE_MIXED_F32, "mixed_f32"),
                       (px.SOLVE_MIXED_BF16, "mixed_bf16")):
        phi = px.alloc_grid(n, torch.float64)
        f = px.alloc_rhs(n, torch.float64)
        f[:, :n] = torch.from_numpy(f_host).cuda()
        st = px.solve(phi, n, f, h, lam, ctx, mode=mode, rtol=1e-10, check_every=2048, raise_on_error=False)
        err = float(np.abs(phi[1:n + 1, 1:n + 1].cpu().numpy() - ex).max() / np.abs(ex).max())
        rec = {"n": n, "mode": name, "status": st.status, "sweeps": st.sweeps, "seconds": round(st.seconds, 3),
               "rel_res_max": st.rel_res_max, "rel_err_vs_exact": err,
               "inner_sweeps": DEFAULT_INNER_SWEEPS.get(name, 0)}
        recs.append(rec)
        log(f"  mixed/{n}: {rec}")
    return recs


def mixed_8192(px, ctx, sweep_ratio):
    """8192^2 (the mixed-precision workload's size), where plain FP64 to the tolerance takes
    hours: measured cost per sweep of each form (the mixed forms including their FP64
    refinement steps at the default inner sweep counts) and residual tracking over the same
    sweeps from phi = 0; the time to the FP64-attainable tolerance is EXTRAPOLATED from the
    slowest mode's closed-form rate and `sweep_ratio` (sweeps to tolerance of each mixed
    form over plain FP64, measured at a smaller size)."""
    import math
    import torch
    import workloads as W
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
    # mixed solves (default inner sweeps) with budgets of 2 and 6 outer steps: the
    # difference gives the time per inner sweep including the FP64 refinement step, without
    # set-up costs
    phi = px.alloc_grid(n, torch.float64)
    f = px.alloc_rhs(n, torch.float64)
    f[:, :n] = torch.from_numpy(f_host).cuda()
    for mode, key in ((px.SOLVE_MIXED_F32, "mixed_f32"), (px.SOLVE_MIXED_BF16, "mixed_bf16")):
        inner = DEFAULT_INNER_SWEEPS[key]
        secs = []
        for steps in (2, 6):
            phi.zero_()
            st = px.solve(phi, n, f, h, lam, ctx, mode=mode, rtol=0.0, max_sweeps=inner * steps,
                          check_every=inner * steps, raise_on_error=False)
            secs.append((st.seconds, st.sweeps))
        per[key] = {"s_per_sweep_incl_refine": (secs[1][0] - secs[0][0]) / (secs[1][1] - secs[0][1]),
                    "inner": inner}
    # the same number of sweeps from phi = 0 in each form: the residuals must track
    track = 32768
    for mode, key in ((px.SOLVE_PLAIN, "plain_f64"), (px.SOLVE_MIXED_F32, "mixed_f32"),
                      (px.SOLVE_MIXED_BF16, "mixed_bf16")):
        phi.zero_()
        st = px.solve(phi, n, f, h, lam, ctx, mode=mode, rtol=0.0, max_sweeps=track, check_every=track,
                      raise_on_error=False)
        per.setdefault("residual_after_%d_sweeps" % track, {})[key] = st.rel_res_max
    del phi, f
    torch.cuda.empty_cache()
    g = slowest_mode_factor(n)
    floor = 5.6e-10  # FP64 attainable relative residual for this field at 8192^2 (exact solution rounded)
    tau = max(1e-10, 4 * floor)
    sweeps = math.log(tau) / math.log(g)
    t_plain = sweeps * per["f64"]["s_per_sweep"]
    for key in ("mixed_f32", "mixed_bf16"):
        per[key]["sweep_ratio_vs_plain"] = sweep_ratio[key]
        per[key]["extrapolated_seconds_to_tau"] = sweeps * sweep_ratio[key] * per[key]["s_per_sweep_incl_refine"]
        per[key]["extrapolated_speedup_vs_plain_f64"] = t_plain / per[key]["extrapolated_seconds_to_tau"]
    per["plain_f64_extrapolated_seconds_to_tau"] = t_plain
    per["tau_eff"] = tau
    per["sweeps_to_tau_closed_form"] = sweeps
    per["note"] = ("extrapolated: per-sweep costs measured at 8192^2, sweep counts from the closed-form rate "
                   "of the slowest mode times the measured mixed/plain sweep ratio")
    log(f"  mixed/8192: {per}")
    return per


def mixed_workload(px, ctx):
    """Mixed-precision refinement (FP32 / BF16 inner sweeps, FP64 outer residual and
    update) against plain FP64 relaxation, on |k|^-2 Gaussian-random-field right-hand
    sides: measured time to 1e-10 at 256^2 and 512^2 (mixed_solves), and the 8192^2
    per-sweep costs with the extrapolated time to tolerance (mixed_8192)."""
    import workloads as W
    out = {"solves": mixed_solves(px, ctx, 256, W.SEED_GRF_8192) + mixed_solves(px, ctx, 512, W.SEED_GRF_8192)}
    at512 = {r["mode"]: r["sweeps"] for r in out["solves"] if r["n"] == 512}
    out["per_sweep_8192"] = mixed_8192(px, ctx, {k: at512[k] / at512["plain_f64"] for k in ("mixed_f32", "mixed_bf16")})
    return out


def _fresh(px, n, f_host):
    import torch
    phi = px.alloc_grid(n, torch.float64)
    f = px.alloc_rhs(n, torch.float64)
    f[:, :n] = torch.from_numpy(f_host).cuda()
    return phi, f


USE_NET = {"nonet": 0, "net": 1, "both": 2}
# (method, smoothing sweeps per step or plain check interval, judge policy)
LEARNED_CONFIGS = (("plain", 1024, None), ("nonet", 64, 2), ("nonet", 64, 1), ("nonet", 16, 2),
                   ("both", 64, 2), ("both", 64, 0), ("both", 16, 1), ("net", 64, 2))


def train_network(px, ctx, train_steps, train_n=1024):
    """The correction network trained on the GPU: (residual, error) pairs of plain solves
    of 8 fields at train_n^2, then train_steps Adam steps on batches of 2.  Returns the
    network and the training record."""
    import torch
    import workloads as W
    from paper_2307_07931_amd import learned
    t0 = time.perf_counter()
    fields = [W.error_field(train_n, W.SEED_TRAIN_BASE + s) for s in range(8)]
    X, T = learned.training_pairs(fields, ctx)
    torch.cuda.synchronize()
    t_pairs = time.perf_counter() - t0
    net = px.Net(W.net_initial_weights(W.SEED_TRAIN_BASE))
    t1 = time.perf_counter()
    hist = learned.train(net, X, T, steps=train_steps, batch=2, lr=2e-3, log_every=max(1, train_steps // 10))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    rec = {"n": train_n, "pairs": int(X.shape[0]), "steps": train_steps, "batch": 2,
           "loss_history": hist, "seconds_pairs": round(t_pairs, 2), "seconds_train": round(t_train, 2)}
    log(f"  learned: {X.shape[0]} pairs in {t_pairs:.1f} s, {train_steps} steps in {t_train:.1f} s, "
        f"loss {hist[0][1]:.3g} -> {hist[-1][1]:.3g}")
    del X, T
    torch.cuda.empty_cache()
    return net, rec


def learned_solve(px, ctx, net, method, n, f_host, smooth, judge, ex=None, rtol=1e-10):
    """One measured solve to max|r| <= rtol max|f| from phi = 0 (plain FP64 relaxation with
    checks every `smooth` sweeps, or the refinement loop without / with the network)."""
    import numpy as np
    phi, f = _fresh(px, n, f_host)
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    if method == "plain":
        st = px.solve(phi, n, f, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=rtol, check_every=smooth,
                      raise_on_error=False)
    else:
        st = px.solve_learned(phi, n, f, h, lam, ctx, net=net, use_net=USE_NET[method], rtol=rtol,
                              smooth_sweeps=smooth, judge=judge, raise_on_error=False)
    rec = {"n": n, "method": method, "smooth": smooth, "judge": judge, "status": st.status, "sweeps": st.sweeps,
           "seconds": round(st.seconds, 4), "rel_res_max": st.rel_res_max}
    if ex is not None:
        rec["rel_err_vs_exact"] = float(np.abs(phi[1:n + 1, 1:n + 1].cpu().numpy() - ex).max() / np.abs(ex).max())
    if method != "plain":
        rec["corrections"], rec["rejected"], rec["fell_back"] = st.corrections, st.rejected, st.fell_back
        rec["discarded_sweeps"] = st.discarded_sweeps
    log(f"  learned/{n}: {rec}")
    return rec


def time_to_tolerance(px, ctx, n=512, train_steps=1000):
    """The metric's second half, measured in the default run: time to max|r| <= 1e-10 max|f|
    at n^2 on an unseen |k|^-2 GRF right-hand side for plain FP64 relaxation, FP64
    refinement around FP32 / BF16 inner sweeps, and the refinement loop without and with
    the network trained here on the GPU; plus the 8192^2 mixed-precision time to the
    FP64-attainable tolerance, EXTRAPOLATED (labelled) from measured per-sweep costs."""
    import workloads as W
    t0 = time.perf_counter()
    out = {"n": n, "rtol": 1e-10, "rhs": f"GRF |k|^-2, seed {W.SEED_EVAL_BASE + 1}"}
    f_host = W.grf_rhs(n, W.SEED_EVAL_BASE + 1)
    ex = exact_solution(f_host)
    solves = mixed_solves(px, ctx, n, W.SEED_EVAL_BASE + 1)
    net, train = train_network(px, ctx, train_steps)
    out["training"] = {k: v for k, v in train.items() if k != "loss_history"}
    for method, smooth, judge in (("nonet", 64, 2), ("net", 64, 2), ("both", 64, 2)):
        solves.append(learned_solve(px, ctx, net, method, n, f_host, smooth, judge, ex=ex))
    net.close()
    out["solves"] = solves
    sec = {r.get("mode") or r["method"]: r["seconds"] for r in solves}
    plain = sec["plain_f64"]
    out["speedup_vs_plain_f64"] = {k: round(plain / v, 3) for k, v in sec.items() if k != "plain_f64"}
    out["network_gain_vs_loop_without"] = round(sec["nonet"] / min(sec["net"], sec["both"]), 3)
    sw = {r.get("mode"): r["sweeps"] for r in solves if r.get("mode")}
    out["mixed_8192_extrapolated"] = mixed_8192(px, ctx, {k: sw[k] / sw["plain_f64"] for k in ("mixed_f32", "mixed_bf16")})
    out["wall_s"] = round(time.perf_counter() - t0, 1)
    return out


def chunked_plain_solve(px, ctx, n, f_host, check_every, chunk_s=20.0, rtol=1e-10):
    """Plain FP64 relaxation to max|r| <= rtol max|f| from phi = 0 in calls of a bounded
    sweep budget (a multiple of check_every, so the residual checks fall on the same sweeps
    as in one call, and the sweep count to tolerance is the same), printing each call's
    progress; seconds and sweeps are summed over the calls."""
    h = 1.0 / n
    lam = OMEGA * h * h / 4.0
    phi, f = _fresh(px, n, f_host)
    # sweeps per call from a short timed call
    st = px.solve(phi, n, f, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=rtol, check_every=check_every,
                  max_sweeps=16 * check_every, raise_on_error=False)
    sweeps, secs = st.sweeps, st.seconds
    budget = max(check_every, int(chunk_s / max(st.seconds / max(st.sweeps, 1), 1e-9)) // check_every * check_every)
    while st.status == px.ENOTCONV:
        st = px.solve(phi, n, f, h, lam, ctx, mode=px.SOLVE_PLAIN, rtol=rtol, check_every=check_every,
                      max_sweeps=budget, raise_on_error=False)
        sweeps += st.sweeps
        secs += st.seconds
        log(f"  plain {n}^2: {sweeps} sweeps, {secs:.1f} s, rel res {st.rel_res_max:.3g}")
    return phi, st.status, sweeps, secs, st.rel_res_max


def learned_workload(px, ctx, train_steps, train_n=1024, eval_n=2048):
    """Learned correction network (4 layers of 3x3 conv, 32 channels, BF16 weights and
    activations, FP32 accumulation) trained on the GPU on (residual, error) pairs of
    plain solves at train_n^2 (initial errors with the |k|^-3 spectrum of L^-1 f for
    |k|^-2 Gaussian-random-field f), then used in the refinement loop (FP64 residual,
    energy-optimal step along the network's direction, plain smoothing sweeps, plain
    relaxation as judge and fallback).  Compared with the same loop without the network
    and with plain FP64 relaxation: measured time to max|r| <= 1e-10 max|f| on unseen
    seeds at 256^2, 512^2 and 1024^2 (every configuration) and at eval_n^2 (plain
    relaxation and the best configuration of each method at 1024^2)."""
    import numpy as np
    import workloads as W
    out = {}
    net, out["training"] = train_network(px, ctx, train_steps, train_n)
    measured = []
    for n in (256, 512, 1024):
        f_host = W.grf_rhs(n, W.SEED_EVAL_BASE + 1)
        ex = exact_solution(f_host)
        tune_sizes(px, ctx, n, f_host, dtypes=("f64",))
        for method, smooth, judge in LEARNED_CONFIGS:
            measured.append(learned_solve(px, ctx, net, method, n, f_host, smooth, judge, ex=ex))
    out["measured"] = measured
    ms = ("plain", "nonet", "net", "both")
    meas = {m: min(r["seconds"] for r in measured if r["method"] == m and r["n"] == 1024) for m in ms}
    out["measured_speedup_vs_plain_1024"] = {m: meas["plain"] / meas[m] for m in ms[1:]}
    # eval_n^2 on an unseen seed: every method measured to the tolerance, each in the
    # configuration that was fastest at 1024^2
    f_host = W.grf_rhs(eval_n, W.SEED_EVAL_BASE)
    ex = exact_solution(f_host)
    tune_sizes(px, ctx, eval_n, f_host, dtypes=("f64",))
    ev = []
    for m in ms:
        best = min((r for r in measured if r["method"] == m and r["n"] == 1024), key=lambda r: r["seconds"])
        if m == "plain":
            phi, status, sweeps, secs, rel = chunked_plain_solve(px, ctx, eval_n, f_host, best["smooth"])
            rec = {"n": eval_n, "method": m, "smooth": best["smooth"], "judge": None, "status": status,
                   "sweeps": sweeps, "seconds": round(secs, 3), "rel_res_max": rel,
                   "rel_err_vs_exact": float(np.abs(phi[1:eval_n + 1, 1:eval_n + 1].cpu().numpy() - ex).max()
                                             / np.abs(ex).max())}
            log(f"  learned/{eval_n}: {rec}")
            del phi
        else:
            rec = learned_solve(px, ctx, net, m, eval_n, f_host, best["smooth"], best["judge"], ex=ex)
        ev.append(rec)
    out["measured_" + str(eval_n)] = ev
    sec = {r["method"]: r["seconds"] for r in ev}
    out["speedup_vs_plain_" + str(eval_n)] = {m: round(sec["plain"] / sec[m], 3) for m in ms[1:]}
    out["network_gain_vs_loop_without_" + str(eval_n)] = round(sec["nonet"] / min(sec["net"], sec["both"]), 3)
    net.close()
    return out


BF16_MFMA_PEAK_TFLOPS = 2500.0
CONV_FLOPS_PER_PIXEL = 2 * 32 * 32 * 9  # one 32 -> 32 layer


def net_workload(px):
    """The correction network's kernels: forward at 1024^2 and 2048^2 (the learned loop's
    per-step cost) and one training evaluation (forward, loss, backward) on 2 x 1024^2,
    timed with HIP events on the stream the kernels run on.  The 32 -> 32 convolutions
    are reported against the dense BF16 matrix-core peak."""
    import torch
    import workloads as W
    net = px.Net(W.net_initial_weights(1))
    out = {}
    for n in (1024, 2048):
        x = torch.from_numpy(W.uniform_rhs(n, 7)).cuda().float().reshape(1, n, n)
        y = torch.empty_like(x)
        t = time_region(lambda: net.forward(x, y), reps=20, warmup=3) / 20
        out[f"forward_{n}"] = {"ms": round(t * 1e3, 4), "gpix_s": round(n * n / t / 1e9, 3),
                               "conv_layers_tflops_if_alone": round(2 * CONV_FLOPS_PER_PIXEL * n * n / t / 1e12, 1)}
        log(f"  net forward {n}^2: {out[f'forward_{n}']}")
        # inference (what the learned loop runs): layers 1 and 2 fused, the same y
        t = time_region(lambda: net.forward(x, y, infer=True), reps=20, warmup=3) / 20
        out[f"infer_{n}"] = {"ms": round(t * 1e3, 4), "gpix_s": round(n * n / t / 1e9, 3)}
        log(f"  net inference {n}^2: {out[f'infer_{n}']}")
    x = torch.from_numpy(W.uniform_rhs(1024, 8)).cuda().float().reshape(1, 1024, 1024).repeat(2, 1, 1).contiguous()
    tg = torch.zeros_like(x)
    t = time_region(lambda: net.loss_grad(x, tg), reps=5, warmup=1) / 5
    out["train_step_2x1024"] = {"ms": round(t * 1e3, 3)}
    log(f"  net training evaluation 2x1024^2: {t * 1e3:.2f} ms")
    net.close()
    return out


def batched_workload(px, ctx, count=512):
    """Batches of uneven problems (sizes drawn from {64,...,1024}, f ~ U[-1,1]): (a) 64
    FP32 sweeps of all `count` problems in one persistent launch per block of sweeps,
    against one px_relax_fused call per problem; (b) FP64 refinement around FP32 sweeps to
    max|r| <= 1e-8 max|f| of ALL `count` problems as graph-replayed batches, against one
    px_solve per problem measured on a sample of each size class and scaled by the class
    counts; every member's error against its exact discrete solution (DST)."""
    import numpy as np
    import torch
    import workloads as W
    sizes = W.batch_sizes(count)
    classes, counts = np.unique(sizes, return_counts=True)
    out = {"count": count, "sizes": {int(k): int(v) for k, v in zip(classes, counts)}}
    items, cells = [], 0
    for i, n in enumerate(sizes):
        n = int(n)
        h = 1.0 / n
        phi = px.alloc_grid(n, torch.float32)
        f = px.alloc_rhs(n, torch.float32)
        f[:, :n] = torch.from_numpy(W.uniform_rhs(n, W.SEED_BATCH_BASE + i)).cuda().float()
        items.append((phi, f, n, h, OMEGA * h * h / 4.0))
        cells += n * n
    sweeps = 64
    t0 = time.perf_counter()
    kb = px.autotune_batched(items, ctx)  # relaxes the problems in place; contents do not matter here
    out["autotune"] = {"k": kb, "seconds": round(time.perf_counter() - t0, 2)}
    log(f"  batched autotune: k={kb} ({out['autotune']['seconds']} s)")
    tb = time_region(lambda: px.relax_batched(items, sweeps, ctx, resmode=px.RES_NONE), reps=3, warmup=1)
    scratch = {}

    def sequential():
        for phi, f, n, h, lam in items:
            if n not in scratch:
                scratch[n] = px.alloc_grid(n, torch.float32)
            px.relax_fused(phi, scratch[n], n, f, h, lam, sweeps, ctx, resmode=px.RES_NONE)
    ts = time_region(sequential, reps=3, warmup=1)
    out["relax"] = {"sweeps": sweeps, "cells": cells, "batched_s": tb / 3, "sequential_s": ts / 3,
                    "batched_gcell_s": cells * sweeps * 3 / tb / 1e9,
                    "sequential_gcell_s": cells * sweeps * 3 / ts / 1e9, "speedup": ts / tb}
    log(f"  batched relax: {out['relax']}")
    del items, scratch
    torch.cuda.empty_cache()

    # (b) the whole batch to 1e-8: FP64 problems, FP32 inner sweeps tuned on the FP32 batch
    # above (the context keeps the batch tuning)
    rtol = 1e-8
    its = []
    for i, n in enumerate(sizes):
        n = int(n)
        h = 1.0 / n
        phi = px.alloc_grid(n, torch.float64)
        f = px.alloc_rhs(n, torch.float64)
        f[:, :n] = torch.from_numpy(W.uniform_rhs(n, W.SEED_BATCH_BASE + i)).cuda()
        its.append((phi, f, n, h, OMEGA * h * h / 4.0))
    # in calls of a bounded budget of inner sweeps (a multiple of the 1024 inner sweeps per
    # FP64 step, so each call ends on a step boundary and the results equal one call's):
    # unconverged problems carry on from their iterate, converged ones drop out
    budget = 1024 * 48
    stats = [None] * count
    todo = list(range(count))
    t_batch, calls = 0.0, 0
    while todo:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        status, st = px.solve_batched([its[i] for i in todo], ctx, mode=px.SOLVE_MIXED_F32, rtol=rtol,
                                      max_sweeps=budget, raise_on_error=False)
        t_batch += time.perf_counter() - t0
        calls += 1
        left = []
        for i, s_ in zip(todo, st):
            prev = stats[i]
            sw = s_.sweeps + (prev.sweeps if prev else 0)
            stats[i] = s_
            stats[i].sweeps = sw
            if s_.rel_res_max > rtol:
                left.append(i)
        if status not in (px.OK, px.ENOTCONV):
            raise RuntimeError(f"batched solve failed: status {status} ({px.last_error()})")
        todo = left
        log(f"  batched solve: {t_batch:.1f} s, {calls} calls, {len(todo)} of {count} problems left")
    # error of every member against its exact discrete solution
    errs = []
    for (phi, f, n, h, lam), i in zip(its, range(count)):
        ex = exact_solution(W.uniform_rhs(n, W.SEED_BATCH_BASE + i))
        errs.append(float(np.abs(phi[1:n + 1, 1:n + 1].cpu().numpy() - ex).max() / np.abs(ex).max()))
    total_sweeps = int(sum(s_.sweeps for s_ in stats))
    solved_cells = int(sum(int(n) * int(n) * s_.sweeps for n, s_ in zip(sizes, stats)))
    # sequential baseline: one px_solve per problem, on the first 2 problems of each class
    seq, same = {}, []
    for c in classes:
        idx = [i for i, n in enumerate(sizes) if n == c][:2]
        tt = []
        for i in idx:
            n = int(c)
            h = 1.0 / n
            phi = px.alloc_grid(n, torch.float64)
            f = px.alloc_rhs(n, torch.float64)
            f[:, :n] = torch.from_numpy(W.uniform_rhs(n, W.SEED_BATCH_BASE + i)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s_ = px.solve(phi, n, f, h, OMEGA * h * h / 4.0, ctx, mode=px.SOLVE_MIXED_F32, rtol=rtol,
                          raise_on_error=False)
            tt.append(time.perf_counter() - t0)
            same.append(bool(torch.equal(phi, its[i][0])))
        seq[int(c)] = sum(tt) / len(tt)
        log(f"  sequential solve {int(c)}^2: {seq[int(c)]:.3f} s per problem (sample of {len(tt)})")
    t_seq = sum(seq[int(c)] * int(k) for c, k in zip(classes, counts))
    by_class = {int(c): max(e for e, n in zip(errs, sizes) if n == c) for c in classes}
    out["solve"] = {"problems": count, "rtol": rtol, "calls": calls, "batched_s": round(t_batch, 2),
                    "sequential_s_scaled": round(t_seq, 2), "sequential_s_per_problem": seq,
                    "speedup": round(t_seq / t_batch, 3), "total_sweeps": total_sweeps,
                    "gcell_updates_s": round(solved_cells / t_batch / 1e9, 1),
                    "max_rel_res": max(s_.rel_res_max for s_ in stats),
                    "sampled_results_identical_to_single_solves": all(same),
                    "max_rel_err_vs_exact_by_size": by_class, "rel_err_vs_exact": [float(f"{e:.3g}") for e in errs]}
    log(f"  batched solve: { {k: v for k, v in out['solve'].items() if k != 'rel_err_vs_exact'} }")
    return out


def boxes_workload(px, ctx):
    """The domain of Section IV split into boxes: 256^2 cells as 4 x 4 boxes of 64^2 (the
    paper's box and domain sizes), 100 sweeps, FP64, Dirichlet edges; ghost layers exchanged
    before every sweep (bit-identical to the whole-domain sweep) or every 4 sweeps, against
    one fused call on the whole 256^2 grid; and 8192^2 as 16 x 16 boxes of 512^2."""
    import numpy as np
    import torch
    import workloads as W
    out = {}
    for nb, n, sweeps in ((4, 64, 100), (16, 512, 96)):
        N = nb * n
        h = 1.0 / N
        lam = OMEGA * h * h / 4.0
        F = W.uniform_rhs(N, 6)
        items = []
        for bi in range(nb):
            for bj in range(nb):
                phi = px.alloc_grid(n, torch.float64)
                f = px.alloc_rhs(n, torch.float64)
                f[:, :n] = torch.from_numpy(np.ascontiguousarray(F[bi * n:(bi + 1) * n, bj * n:(bj + 1) * n])).cuda()
                items.append((phi, f, n, h, lam))
        rec = {"domain": N, "boxes": f"{nb}x{nb} of {n}^2", "sweeps": sweeps}
        for ex in (1, 4, 8):
            if sweeps % ex:
                continue
            t = time_region(lambda: px.relax_boxes(items, nb, nb, sweeps, ctx, exchange=ex), reps=3, warmup=1) / 3
            rec[f"exchange_{ex}_ms"] = round(t * 1e3, 3)
            rec[f"exchange_{ex}_gcell_s"] = round(N * N * sweeps / t / 1e9, 2)
        d = {"phi0": px.alloc_grid(N, torch.float64), "phi_out": px.alloc_grid(N, torch.float64),
             "f": px.alloc_rhs(N, torch.float64), "n": N, "h": h, "lam": lam}
        d["f"][:, :N] = torch.from_numpy(F).cuda()
        t = time_region(lambda: px.relax_fused(d["phi0"], d["phi_out"], N, d["f"], h, lam, sweeps, ctx,
                                               resmode=px.RES_NONE), reps=3, warmup=1) / 3
        rec["whole_grid_ms"] = round(t * 1e3, 3)
        rec["whole_grid_gcell_s"] = round(N * N * sweeps / t / 1e9, 2)
        log(f"  boxes: {rec}")
        out[f"{N}"] = rec
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
    ap.add_argument("--workload", choices=["relax", "mixed", "learned", "batched", "net", "boxes"], default="relax",
                    help="relax: the fused relaxation benchmark (default); mixed: mixed-precision "
                         "refinement against plain FP64 (time to tolerance); learned: the trained "
                         "correction network in the refinement loop; batched: 512 uneven problems")
    ap.add_argument("--train-steps", type=int, default=1000)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--cpu-sweeps", type=int, default=SWEEPS)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); sharding the relaxation over "
              f"GPUs (box decomposition) is designed but not implemented", file=sys.stderr)
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
                          "value": round(p8["mixed_f32"]["extrapolated_speedup_vs_plain_f64"], 3),
                          "unit": "x time-to-tolerance speedup (mixed FP32 vs plain FP64, 8192^2, extrapolated)",
                          "higher_is_better": True, "n_gpus": 1, "data": "synthetic", "results": res,
                          "wall_s": round(time.perf_counter() - t0, 1)}), flush=True)
        ctx.close()
        return

    if args.workload in ("learned", "batched", "net", "boxes"):
        t0 = time.perf_counter()
        if args.workload == "boxes":
            res = boxes_workload(px, ctx)
            value, unit = res["256"]["exchange_1_gcell_s"], "Gcell-updates/s (256^2 as 4 x 4 boxes of 64^2, exchange every sweep)"
        elif args.workload == "net":
            res = net_workload(px)
            value, unit = res["infer_2048"]["gpix_s"], "Gpixel/s (network inference, 2048^2)"
        elif args.workload == "learned":
            res = learned_workload(px, ctx, args.train_steps)
            value = max(res["speedup_vs_plain_2048"]["net"], res["speedup_vs_plain_2048"]["both"])
            unit = "x time-to-1e-10 speedup (learned loop with the network vs plain FP64, 2048^2, measured)"
        else:
            res = batched_workload(px, ctx)
            value, unit = res["solve"]["speedup"], "x speedup (one batched solve vs per-problem solves)"
        print(json.dumps({"metric": METRIC, "workload": args.workload, "value": round(value, 3), "unit": unit,
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
                "frac": round(achieved / HBM_PEAK_GBS, 4), "alg_bytes_per_launch": BYTES_PER_CELL["f64"] * N * N,
                # what a kernel doing one sweep per pass over HBM would have to move for
                # this throughput (24 B per cell-update)
                "sweep_equivalent_GBs": round(BYTES_PER_CELL["f64"] * value, 1),
                "sweep_equivalent_frac": round(BYTES_PER_CELL["f64"] * value / HBM_PEAK_GBS, 3)}
    tr = measured_traffic(tb, rows)
    traffic = round(tr["read"] + tr["write"]) if tr else None
    if tr:
        hbm_view["traffic_read"] = round(tr["read"])
        hbm_view["traffic_write"] = round(tr["write"])
        hbm_view["traffic_over_algorithmic"] = round((tr["read"] + tr["write"]) / hbm_view["alg_bytes_per_launch"], 3)
        hbm_view["actual_GBs"] = round((tr["read"] + tr["write"]) / per_launch_s / 1e9, 1)
        if "memory_side" in tr:
            ms_ = tr["memory_side"]
            hbm_view["memory_side_read"] = ms_["read"]
            hbm_view["memory_side_write"] = ms_["write"]
    # roofline: arithmetic intensity of a launch (k sweeps: 9k FLOP per 24 B of HBM traffic
    # per cell) against the ridge point of the no-FMA FP64 peak over the HBM peak; below
    # the ridge (every k <= 8: at most 3 FLOP/B against 4.9) the HBM roof binds
    tflops = FLOPS_PER_CELL_SWEEP * N * N * tb / per_launch_s / 1e12
    intensity = FLOPS_PER_CELL_SWEEP * tb / BYTES_PER_CELL["f64"]
    ridge = FP64_NOFMA_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    alu_view = {"achieved": round(tflops, 3), "peak": round(FP64_NOFMA_PEAK_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(tflops / FP64_NOFMA_PEAK_TFLOPS, 4),
                "alg_flops_per_launch": FLOPS_PER_CELL_SWEEP * N * N * tb}
    if intensity < ridge:
        roofline = {"bound": "hbm", **hbm_view, "traffic": traffic, "alu_view": alu_view}
    else:
        roofline = {"bound": "alu", **{k: v for k, v in alu_view.items()}, "traffic": traffic, "hbm_view": hbm_view}
    roofline["intensity_flop_per_byte"] = round(intensity, 3)
    roofline["ridge_flop_per_byte"] = round(ridge, 3)
    roofline["kernel"] = f"relax_tb_kernel<double,2,{tb},*> ({rows or 'default'} rows per tile)"

    var = None if args.no_variants else variants(px, ctx, norms)
    cpu = None if args.no_cpu else cpu_baseline(args.cpu_sweeps)
    ttt = None if args.no_ttt else time_to_tolerance(px, ctx)

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
        "time_to_tolerance": ttt,
    }
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()

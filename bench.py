"""Benchmark: filter throughput and time-to-residual of the R-ChFSI hot path on one MI355X.

Workload (default): dense generalized pencil, N = 8192, block 320, 256 wanted,
Chebyshev degree 20, B = D + eps S with ||D^{-1} eps S||_2 = 0.05, approximate
inverse D^{-1}; synthetic seeded inputs from ``workloads`` (seed 1001, start
block seed 2001).  One step = one outer iteration of Algorithm 1 with the
residual filter (Algorithm 3) in FP32 on MFMA followed by the FP64 CholQR /
Rayleigh-Ritz / residual-norm pass, all through the C ABI.

Prints ONE JSON line.  ``value`` is the filter's algorithmic throughput
(2 N^2 b flops per recurrence step) over the filter time of the timed steps.
Extras: the dominant kernel's roofline entry (HIP events around each FP32
GEMM launch), the CPU oracle timed on a bounded sample, and time-to-residual
of FP32 R-ChFSI vs the FP64 baselines.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "filter GFLOP/s + time-to-residual 1e-8, FP64 ChFSI vs FP32/BF16 R-ChFSI; p99 lat"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_MFMA_TFLOPS = 78.6
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# HBM bytes per FP32 filter step at N = 8192, b = 320: the GEMM (64x64x32
# tiles, split-K 8) plus the split-K reduction that carries the three-term
# epilogue, the two kernels the step's timing brackets.  FETCH_SIZE and
# WRITE_SIZE from two rocprofv3 counter passes over this script, scaled by what
# the same counters read for a 1 GiB device copy (FETCH x 2.000, WRITE x 1.000);
# summary under profiles/.  Other shapes report null.
TRAFFIC_F32_FILTER_STEP = {(8192, 320): 511.5e6}
# the same for the BF16-product step (product, split-K reduction that also
# rounds the next step's operand; the rounding pass of a filter's first step
# averaged over its 19 steps: profiles/dense_n8192_b320_bf16_wide_step_traffic.md)
TRAFFIC_BF16_FILTER_STEP = {(8192, 320): 277.2e6}
# the same for the BF16 z-march filter step on the 128^3 grid (block 1200) and
# the 160^3 grid (block 2400)
TRAFFIC_ZMARCH = {(128, 1200, "bf16"): 21.98e9, (160, 2400, "bf16"): 89.61e9}
# HBM bytes per Bloch filter step at 128^3 x 600 complex vectors (BF16): the
# corrected z-march plus the boundary-correction kernel (two counter passes,
# profiles/grid_128_b600_bloch_bf16_step_traffic.md)
TRAFFIC_BLOCH_STEP = {(128, 600, "bf16"): 24.18e9}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--block", type=int, default=320)
    ap.add_argument("--wanted", type=int, default=256)
    ap.add_argument("--degree", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-solve", type=str, default="",
                    help="comma list of cfg0,cfg1: also time full CPU oracle solves at full size")
    ap.add_argument("--no-extras", action="store_true", help="skip time-to-residual runs")
    ap.add_argument("--dense-prec", choices=("fp32", "bf16"), default="fp32",
                    help="dense workload: precision of the timed residual-filter steps (the "
                         "metric is quoted on FP32; bf16 times the bfloat16-product filter)")
    ap.add_argument("--no-grid", action="store_true",
                    help="dense workload: skip the 128^3 grid extra")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", choices=("dense", "grid", "serving"), default="dense",
                    help="dense: the headline line; grid / serving: extra measurement lines")
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--bloch", type=str, default="",
                    help="kx,ky,kz: the grid pencil at this wave vector (complex, Section 4.3), "
                         "half the block in complex vectors")
    ap.add_argument("--wells", type=int, default=64)
    ap.add_argument("--prec", choices=("bf16", "fp32", "fp64"), default="bf16")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--sequences", type=int, default=64)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--sizes", type=str, default="512,1024,2048,4096,8192")
    ap.add_argument("--ttr", action="store_true",
                    help="grid workload: also run solves to residual 1e-8 (reduced precision "
                         "R-ChFSI, FP64 R-ChFSI, FP64 ChFSI with D^-1 = I)")
    ap.add_argument("--ttr-iters", type=int, default=120)
    ap.add_argument("--ttr-chfsi-iters", type=int, default=25)
    ap.add_argument("--ttr-runs", type=str, default="",
                    help="grid workload: comma list of time-to-residual runs to do (names as "
                         "in the output: <prec>_rchfsi, fp64_rchfsi, fp64_chfsi_dinv_identity); "
                         "default all")
    ap.add_argument("--ttr-memory-mode", type=int, default=-1,
                    help="grid workload: force memory_mode of the reduced-precision "
                         "time-to-residual run (-1: by free memory)")
    ap.add_argument("--ttr-escalate", type=int, default=0,
                    help="grid workload: > 0 lets the BF16 time-to-residual run switch to FP32 "
                         "after this many passes without a new lowest max residual")
    ap.add_argument("--fp64-panel", type=int, default=600,
                    help="grid workload: column panel for the FP64 R-ChFSI filter timing when "
                         "the full FP64 solve does not fit in device memory")
    return ap.parse_args()


def host_info():
    """CPU model and the BLAS library NumPy dispatches to, for the CPU baselines."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    blas = {"library": "unknown", "threads": None}
    try:
        from threadpoolctl import threadpool_info
        for i in threadpool_info():
            if i.get("user_api") == "blas":
                blas = {"library": f"{i.get('internal_api')} {i.get('version')}",
                        "arch": i.get("architecture"), "threads": i.get("num_threads")}
                break
    except ImportError:
        pass
    return {"cpu_model": model, "blas": blas}


def cpu_baseline(prob, X0, seconds_target=20.0):
    """Time the CPU oracle's residual filter (Algorithm 3, FP64 NumPy) on a column sample."""
    import numpy as np
    from oracle import filters, rr
    n = prob.n
    hinfo = host_info()
    cores = hinfo["blas"]["threads"] or len(os.sched_getaffinity(0))
    bcols = min(prob.block, 80)
    Xs = np.ascontiguousarray(X0[:, :bcols])
    o = rr.rayleigh_ritz(Xs, filters.dense_op(prob.A), filters.dense_op(prob.B))
    lam = o["lam"]
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), prob.meta["lmax"], lam[-1])
    p = prob.degree
    t0 = time.perf_counter()
    reps = 0
    while True:
        filters.residual_filter(filters.dense_op(prob.A), filters.diag_op(prob.dinv), o["X"], lam,
                                o["R"], p, *bounds)
        reps += 1
        if time.perf_counter() - t0 > seconds_target or reps >= 5:
            break
    dt = (time.perf_counter() - t0) / reps
    flops = 2.0 * n * n * bcols * (p - 1)
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": cores, "kind": "oracle",
            **hinfo,
            "sample": f"Algorithm 3 FP64 NumPy filter, N={n}, {bcols} of {prob.block} columns "
                      f"(the filter is column-independent), degree {p}, {reps} pass(es), "
                      f"{dt:.2f} s per pass"}


def cpu_solve_times(configs=("cfg0", "cfg1"), max_iter=60):
    """Full solves of the CPU oracle (Algorithm 1, FP64 NumPy) at full size.

    cfg0: dense standard N = 1024, 32 wanted, block 40, degree 16, tolerance 1e-10.
    cfg1: dense generalized N = 8192, 256 wanted, block 320, degree 20, tolerance 1e-8;
    R-ChFSI with the approximate inverse D^{-1}, and ChFSI with the exact B^{-1}
    (Cholesky solves), the paper's FP64 baseline.  lambda_max comes from 12 oracle
    Lanczos steps (Section 2.1's estimate), included in the time, as the GPU
    solves estimate it inside the library.  Same seeded inputs as the GPU runs."""
    import numpy as np
    import scipy.linalg as sla
    import workloads as wl
    from oracle import bounds as obounds
    from oracle import filters, solver
    hinfo = host_info()
    res = {"kind": "oracle", **hinfo,
           "cores": hinfo["blas"]["threads"] or len(os.sched_getaffinity(0))}
    for cfg in configs:
        if cfg == "cfg0":
            p = wl.dense_standard(n=1024, n_low=32, block=40, degree=16, seed=1000)
            B = None
            tol = 1e-10
            runs = (("fp64_rchfsi", "rchfsi"), ("fp64_chfsi", "chfsi"))
        else:
            p = wl.dense_generalized(n=8192, n_low=256, block=320, degree=20, seed=1001)
            B = p.B
            tol = 1e-8
            runs = (("fp64_rchfsi", "rchfsi"), ("fp64_chfsi", "chfsi"))
        X0 = wl.random_block(p.n, p.block, 2001)
        nw = p.n_wanted
        apply_A = filters.dense_op(p.A)
        out = {"n": p.n, "block": p.block, "wanted": nw, "degree": p.degree, "tol": tol}
        for label, method in runs:
            t0 = time.perf_counter()
            if B is None:
                apply_B = filters.identity_op()
                dinv_op = filters.identity_op()
                solve_B = lambda y: y
            else:
                apply_B = filters.dense_op(B)
                cf = sla.cho_factor(B)
                solve_B = lambda y, cf=cf: sla.cho_solve(cf, y)
                dinv_op = (filters.diag_op(p.dinv) if method == "rchfsi"
                           else (lambda V, cf=cf: sla.cho_solve(cf, V)))
            v0 = wl.random_block(p.n, 1, 5)[:, 0]
            est = obounds.lanczos_bounds(lambda x: p.A @ x, lambda x: apply_B(x[:, None])[:, 0],
                                         solve_B, v0, 12)
            r = solver.solve(apply_A, apply_B, dinv_op, X0, nw, p.degree, tol, max_iter,
                             ("ritz", est["upper"]), method=method)
            dt = time.perf_counter() - t0
            out[label] = {"seconds": round(dt, 2), "iterations": int(r["iters"]),
                          "converged": bool(r["converged"]),
                          "max_res": float(np.max(r["resnorm"][:nw]))}
            log(f"CPU oracle {cfg} {label}: {dt:.1f} s, {r['iters']} iterations, "
                f"converged {r['converged']}")
        res[cfg] = out
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for {args.gpus}); "
              f"multi-GPU sharding is not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "grid":
        return bench_grid(args)
    if args.workload == "serving":
        return bench_serving(args)
    import numpy as np
    import torch

    import paper_2503_22652_amd as P
    import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    n, b, nw, p = args.n, args.block, args.wanted, args.degree
    t_gen = time.perf_counter()
    prob = wl.dense_generalized(n=n, n_low=nw, block=b, degree=p, seed=1001)
    X0 = wl.random_block(n, b, 2001)
    log(f"inputs generated in {time.perf_counter() - t_gen:.1f} s")

    A = P.to_colmajor(prob.A)
    B = P.to_colmajor(prob.B)
    d = torch.from_numpy(prob.dinv).cuda()
    opA, opB = P.dense_operator(A), P.dense_operator(B)
    stream = torch.cuda.current_stream()

    def ctx_for(method, prec, profile=0, max_iter=60, tol=1e-8, binv_exact=0,
                lambda_max=math.nan):
        # lambda_max = NaN: chfsi_solve makes the Lanczos estimate (included in
        # its time)
        prm = P.make_params(nw, b, p, max_iter=max_iter, tol=tol, method=method,
                            filter_prec=prec, lambda_max=lambda_max, profile=profile,
                            binv_exact=binv_exact)
        return P.chfsi_create(opA, opB, d, prm, stream=stream, keep=(A, B, d))

    # ------------------------------------------------------------------
    # timed steps: FP32 R-ChFSI outer iterations (filter + RR + residuals)
    # ------------------------------------------------------------------
    dprec = P.PREC_BF16 if args.dense_prec == "bf16" else P.PREC_FP32
    peak = PEAK_BF16_MFMA_TFLOPS if args.dense_prec == "bf16" else PEAK_FP32_MFMA_TFLOPS
    ctx = ctx_for(P.METHOD_RCHFSI, dprec, profile=1)
    # lambda_max for the explicit filter calls: the library's Lanczos estimate
    torch.cuda.synchronize()
    t_b = time.perf_counter()
    _, lmax, _, lmax_ritz = P.chfsi_estimate_bounds(ctx)
    bounds_ms = (time.perf_counter() - t_b) * 1e3
    prob.meta["lmax"] = lmax
    log(f"lambda_max estimate {lmax:.6g} (top Ritz value {lmax_ritz:.6g}) in {bounds_ms:.1f} ms")
    X = P.to_colmajor(X0)
    Y = P.colmajor_empty(n, b)
    R = P.colmajor_empty(n, b)
    Xn = P.colmajor_empty(n, b)
    ritz, norms = P.chfsi_rayleigh_ritz(ctx, X, Xn, R)
    X, Xn = Xn, X

    filt_ev = []

    def step():
        nonlocal X, Xn, ritz, norms
        e1, eb = ritz[0], ritz[-1]
        lmin, lT = e1 - 0.05 * (eb - e1), eb
        s0 = torch.cuda.Event(enable_timing=True)
        s1 = torch.cuda.Event(enable_timing=True)
        s0.record(stream)
        P.chfsi_filter(ctx, X, ritz, R, Y, lmin, lmax, lT)
        s1.record(stream)
        filt_ev.append((s0, s1))
        ritz, norms = P.chfsi_rayleigh_ritz(ctx, Y, X, R)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    P.chfsi_filter_kernel_time(ctx)          # discard warm-up kernel times
    filt_ev.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms, kern_n = P.chfsi_filter_kernel_time(ctx)
    filt_ms = sum(a.elapsed_time(b_) for a, b_ in filt_ev)
    step_flops = 2.0 * n * n * b * (p - 1)
    value = step_flops * args.steps / (filt_ms / 1e3) / 1e9
    per_launch_ms = kern_ms / max(kern_n, 1)
    achieved_tflops = 2.0 * n * n * b / (per_launch_ms / 1e3) / 1e12
    max_res_after = max(norms[:nw])
    log(f"steps: wall {wall * 1e3 / args.steps:.2f} ms/step, filter {filt_ms / args.steps:.2f} "
        f"ms/step, GEMM {per_launch_ms:.3f} ms/launch over {kern_n} launches, "
        f"max residual {max_res_after:.2e}")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.dense_prec == "fp32" else "bf16 products, f32 blocks",
        "data": "synthetic",
        "config": {
            "workload": f"dense generalized A x = lambda B x, N={n}, block {b}, {nw} wanted, "
                        f"degree {p}; FP32 R-ChFSI filter (MFMA) + FP64 CholQR/Rayleigh-Ritz/"
                        f"residual norms; ||D^-1 eps S||_2=0.05",
            "n": n, "block": b, "n_wanted": nw, "degree": p,
            "lambda_max_estimate": round(lmax, 6), "bounds_estimate_ms": round(bounds_ms, 1),
            "filter_ms_per_step": round(filt_ms / args.steps, 3),
        },
        "roofline": {
            "bound": "mfma",
            "achieved": round(achieved_tflops, 2),
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / peak, 4),
            "traffic": (TRAFFIC_F32_FILTER_STEP if args.dense_prec == "fp32"
                        else TRAFFIC_BF16_FILTER_STEP).get((n, b)),
            "traffic_unit": "bytes per launch",
            "kernel": ("gemm_kernel<float> + splitk_reduce4_kernel (FP32 residual-filter step, "
                       "2*N^2*b flops per launch)") if args.dense_prec == "fp32" else
                      ("gemm_bf16_wide_kernel + splitk_reduce4_kernel, which also rounds the "
                       "next step's operand (k_scale_bf16 on a filter's first step) (BF16-product "
                       "residual-filter step, 2*N^2*b flops per launch)"),
            "ms_per_launch": round(per_launch_ms, 4),
        },
    }

    # ------------------------------------------------------------------
    # extras: time to residual 1e-8 (FP32/BF16/FP64 R-ChFSI, the plain FP64
    # filter with the exact inverse B^{-1}) and the plain FP64 filter with
    # D^{-1} (stagnation floor; its filter rate)
    # ------------------------------------------------------------------
    if not args.no_extras:
        ttr = {}
        for name, method, prec, iters in (("fp32_rchfsi", P.METHOD_RCHFSI, P.PREC_FP32, 60),
                                          ("bf16_rchfsi", P.METHOD_RCHFSI, P.PREC_BF16, 60),
                                          ("fp64_rchfsi", P.METHOD_RCHFSI, P.PREC_FP64, 60),
                                          ("fp64_chfsi_exact", P.METHOD_CHFSI, P.PREC_FP64, 60),
                                          ("fp64_chfsi_dinv", P.METHOD_CHFSI, P.PREC_FP64, 15)):
            exact = name == "fp64_chfsi_exact"
            torch.cuda.synchronize()
            t0c = time.perf_counter()
            c2 = ctx_for(method, prec, profile=1, max_iter=iters, binv_exact=int(exact))
            torch.cuda.synchronize()
            create_s = time.perf_counter() - t0c
            Xs = P.to_colmajor(X0)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st, ev, rn, rep = P.chfsi_solve(c2, Xs)
            dt = time.perf_counter() - t1
            fl_rate = rep["filter_flops"] / max(rep["time_filter_ms"], 1e-9) / 1e6
            ttr[name] = {"status": P.STATUS_NAMES[st], "seconds": round(dt, 3),
                         "iterations": rep["iterations"],
                         "max_residual": rep["max_residual"],
                         "filter_gflops": round(fl_rate, 1),
                         "filter_ms": round(rep["time_filter_ms"], 2),
                         "rr_ms": round(rep["time_rr_ms"], 2),
                         "bounds_ms": round(rep["time_bounds_ms"], 1),
                         "jacobi_sweeps": rep["jacobi_sweeps"]}
            if exact:
                # B^{-1} A formed once in chfsi_create (not in seconds above)
                ttr[name]["setup_seconds"] = round(create_s, 3)
            if rep["kernel_launches"]:
                ttr[name]["product_ms_per_launch"] = round(rep["kernel_ms"] / rep["kernel_launches"], 4)
                ttr[name]["product_tflops"] = round(
                    2.0 * n * n * b / (rep["kernel_ms"] / rep["kernel_launches"] / 1e3) / 1e12, 1)
            log(name, ttr[name])
            del c2, Xs
        for lo in ("fp32", "bf16"):
            if ttr[lo + "_rchfsi"]["status"] == "OK" and ttr["fp64_rchfsi"]["status"] == "OK":
                ttr[f"speedup_{lo}_vs_fp64_rchfsi"] = round(
                    ttr["fp64_rchfsi"]["seconds"] / ttr[lo + "_rchfsi"]["seconds"], 3)
            if ttr[lo + "_rchfsi"]["status"] == "OK" and ttr["fp64_chfsi_exact"]["status"] == "OK":
                ttr[f"speedup_{lo}_vs_fp64_chfsi_exact"] = round(
                    ttr["fp64_chfsi_exact"]["seconds"] / ttr[lo + "_rchfsi"]["seconds"], 3)
        ttr["fp64_chfsi_filter_vs_fp32_rchfsi_filter_rate"] = round(
            ttr["fp32_rchfsi"]["filter_gflops"] / max(ttr["fp64_chfsi_dinv"]["filter_gflops"], 1e-9), 3)
        out["time_to_residual"] = ttr
        out["paper_context"] = ("paper reports up to 2.7x filtering / 2.1x eigensolve speedup "
                                "(TF32B vs FP64 R-ChFSI, complex Hermitian) on Intel Data Center "
                                "GPU Max (Aurora); context only")
        out["complex_hermitian_filter"] = complex_filter_rates(P, n, b, nw, p, stream)

    if args.calibrate_copy:
        nbytes = args.calibrate_copy * (1 << 20)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nbytes

    if not args.no_cpu_baseline:
        log("timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(prob, X0)
    if args.cpu_solve:
        out["cpu_solve"] = cpu_solve_times(tuple(c for c in args.cpu_solve.split(",") if c))

    # ------------------------------------------------------------------
    # grid extra: the 128^3 x 1200 BF16 grid pencil (HBM-bound stencil
    # filter), two timed outer iterations, its roofline and CPU baseline
    # ------------------------------------------------------------------
    if not args.no_grid:
        del ctx, X, Xn, Y, R
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        gout, S = grid_steps(128, 64, "bf16", "", steps=2, warmup=1)
        out["grid"] = {k: gout[k] for k in ("value", "unit", "ms_per_step", "steps", "warmup",
                                            "dtype", "config", "roofline")}
        if not args.no_cpu_baseline:
            log("timing the CPU oracle (C/OpenMP grid filter) ...")
            out["grid"]["cpu_baseline"] = grid_cpu_baseline(S["prob"])
        log("grid", out["grid"]["value"], out["grid"]["roofline"])
    print(json.dumps(out), flush=True)


def complex_filter_rates(P, n, b, nw, p, stream):
    """Complex Hermitian counterpart of the dense workload (device-built: complex
    reflectors, complex Hermitian S, real D): one residual-filter pass of degree
    p in FP64, FP32 and BF16 products (8 n^2 b flops per step), and the time to
    max residual 1e-8 of full solves in each."""
    import numpy as np
    import torch
    from workloads.gpu import hermitian_problem
    A, B, dinv, _ = hermitian_problem(n, nw, seed=1003)
    # lambda_max: the library's Lanczos estimate on a first context
    c0 = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), dinv,
                        P.make_params(nw, b, p, method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64),
                        stream=stream, keep=(A, B, dinv))
    lmax = P.chfsi_estimate_bounds(c0)[1]
    del c0
    g = torch.Generator(device="cuda")
    g.manual_seed(2003)
    X = torch.complex(torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g),
                      torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g)).t()
    R = (1e-3 * torch.complex(torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g),
                              torch.randn((b, n), dtype=torch.float64, device="cuda",
                                          generator=g))).t()
    lam = np.sort(np.random.default_rng(2003).uniform(-1.0, 0.2, b))
    bounds = (lam[0] - 0.05 * (lam[-1] - lam[0]), lmax, lam[-1])
    Y = P.colmajor_empty_complex(n, b)
    step_flops = 8.0 * n * n * b
    res = {"workload": f"complex Hermitian A x = lambda B x, N={n}, block {b}, {nw} wanted, "
                       f"degree {p}, ||D^-1 eps S||_2=0.05"}
    for name, prec in (("fp64", P.PREC_FP64), ("fp32", P.PREC_FP32), ("bf16", P.PREC_BF16)):
        prm = P.make_params(nw, b, p, method=P.METHOD_RCHFSI, filter_prec=prec, lambda_max=lmax,
                            profile=1)
        ctx = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), dinv, prm,
                             stream=stream, keep=(A, B, dinv))
        P.chfsi_filter(ctx, X, lam, R, Y, *bounds)
        torch.cuda.synchronize()
        P.chfsi_filter_kernel_time(ctx)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(3):
            P.chfsi_filter(ctx, X, lam, R, Y, *bounds)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        kms, kn = P.chfsi_filter_kernel_time(ctx)
        per = kms / max(kn, 1)
        res[name] = {"filter_ms": round(ms, 3),
                     "filter_tflops": round(step_flops * (p - 1) / (ms / 1e3) / 1e12, 1),
                     "product_ms_per_launch": round(per, 4),
                     "product_tflops": round(step_flops / (per / 1e3) / 1e12, 1)}
        log("complex", name, res[name])
        del ctx
    for lo in ("fp32", "bf16"):
        res[f"filter_speedup_{lo}_vs_fp64"] = round(res["fp64"]["filter_ms"] / res[lo]["filter_ms"], 3)
    # time to max residual 1e-8 over the nw wanted pairs, from one random start
    X0 = torch.complex(torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g),
                       torch.randn((b, n), dtype=torch.float64, device="cuda", generator=g)).t()
    ttr = {}
    for name, prec in (("fp64", P.PREC_FP64), ("fp32", P.PREC_FP32), ("bf16", P.PREC_BF16)):
        prm = P.make_params(nw, b, p, max_iter=60, tol=1e-8, method=P.METHOD_RCHFSI,
                            filter_prec=prec)      # lambda_max estimated inside the solve
        ctx = P.chfsi_create(P.hermitian_operator(A), P.hermitian_operator(B), dinv, prm,
                             stream=stream, keep=(A, B, dinv))
        Xs = X0.t().clone().t()   # a fresh copy: the solve overwrites its block
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, ev, rn, rep = P.chfsi_solve(ctx, Xs)
        dt = time.perf_counter() - t1
        ttr[name] = {"status": P.STATUS_NAMES[st], "seconds": round(dt, 3),
                     "iterations": rep["iterations"], "max_residual": rep["max_residual"],
                     "filter_ms": round(rep["time_filter_ms"], 2),
                     "rr_ms": round(rep["time_rr_ms"], 2)}
        log("complex solve", name, ttr[name])
        del ctx, Xs
    for lo in ("fp32", "bf16"):
        if ttr[lo]["status"] == "OK" and ttr["fp64"]["status"] == "OK":
            ttr[f"speedup_{lo}_vs_fp64"] = round(ttr["fp64"]["seconds"] / ttr[lo]["seconds"], 3)
    res["time_to_residual"] = ttr
    res["lambda_max_estimate"] = round(lmax, 6)
    return res


def grid_steps(g, wells, prec_name, bloch, steps, warmup, degree=None):
    """Timed outer iterations (filter + FP64 Rayleigh-Ritz) of the grid pencil
    (periodic 27-point Q1 FE stencils + Gaussian wells) with the residual filter
    in BF16 (or FP32/FP64) storage, through chfsi_solve.  lambda_max is the
    library's Lanczos estimate (chfsi_estimate_bounds), made once before the
    timed steps.  Returns (out dict, state for the time-to-residual runs)."""
    import numpy as np
    import torch

    import paper_2503_22652_amd as P
    import workloads as wl

    torch.cuda.set_device(0)
    b = {128: 1200, 160: 2400}.get(g, max(16, (g * g) // 12))
    nw = int(round(b / 1.2)) if g not in (128, 160) else {128: 1000, 160: 2000}[g]
    p = degree if degree else {160: 40}.get(g, 30)
    prob = wl.stencil_problem(grid=g, n_wells=wells, n_wanted=nw, block=b, degree=p,
                              seed=1002 if g != 160 else 1004)
    n = prob.n
    kvec = tuple(float(v) for v in bloch.split(",")) if bloch else None
    if kvec is not None:
        # complex vectors: b planar columns = b / 2 complex vectors
        b, nw = b // 2, nw // 2
    prec = {"bf16": P.PREC_BF16, "fp32": P.PREC_FP32, "fp64": P.PREC_FP64}[prec_name]
    esize = {"bf16": 2, "fp32": 4, "fp64": 8}[prec_name]
    Vd = torch.from_numpy(np.ascontiguousarray(prob.V).reshape(-1)).cuda()
    opA = P.stencil_operator(prob.shape, prob.coef_A, coef_mass=prob.coef_B, field=Vd,
                             field_mode=prob.field_mode, bloch=kvec)
    opB = P.stencil_operator(prob.shape, prob.coef_B, bloch=kvec)
    torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    mode = 0
    prm = P.make_params(nw, b, p, max_iter=warmup, tol=0.0, method=P.METHOD_RCHFSI,
                        filter_prec=prec, profile=1, seed=2002, init_random=1)
    cw = 2 if kvec is not None else 1          # planar columns per vector
    need = P.chfsi_workspace_bytes(opA, opB, prm) + n * b * 8 * cw
    if need > 0.9 * free and prec != P.PREC_FP64 and kvec is None:
        mode = 1
    prm.memory_mode = mode
    log(f"grid {g}^3: n={n}, b={b}, p={p}, memory_mode={mode}, "
        f"workspace {P.chfsi_workspace_bytes(opA, opB, prm) / 2**30:.1f} GiB")
    stream = torch.cuda.current_stream()
    ctx = P.chfsi_create(opA, opB, None, prm, stream=stream, keep=(Vd,))
    torch.cuda.synchronize()
    tb = time.perf_counter()
    lo_est, lmax, th_min, th_max = P.chfsi_estimate_bounds(ctx)
    bounds_ms = (time.perf_counter() - tb) * 1e3
    log(f"lambda_max estimate {lmax:.6g} (Ritz {th_max:.6g}) in {bounds_ms:.0f} ms")
    X = P.colmajor_empty(n, b) if kvec is None else P.colmajor_empty_complex(n, b)
    if warmup > 0:
        prm.lambda_max = lmax
        ctx.close()
        ctx = P.chfsi_create(opA, opB, None, prm, stream=stream, keep=(Vd,))
        P.chfsi_solve(ctx, X)                      # random start + warm-up iterations
    P.chfsi_filter_kernel_time(ctx)
    prm2 = P.make_params(nw, b, p, max_iter=steps, tol=0.0, method=P.METHOD_RCHFSI,
                         filter_prec=prec, lambda_max=lmax, profile=1, seed=2002,
                         init_random=0 if warmup > 0 else 1, memory_mode=mode)
    ctx.close()
    ctx = P.chfsi_create(opA, opB, None, prm2, stream=stream, keep=(Vd,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st, ev, rn, rep = P.chfsi_solve(ctx, X)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    its = max(rep["iterations"], 1)
    per = rep["kernel_ms"] / max(rep["kernel_launches"], 1)
    # algorithmic bytes of one filter step: four streams over the n x (cw b)
    # planar block; a Bloch step adds the boundary pass (read the wrapped
    # neighbours' source values once, read and write the output there)
    nbnd = n - (g - 2) ** 3 if kvec is not None else 0
    launch_bytes = 4.0 * esize * n * b * cw + 3.0 * esize * nbnd * b * cw
    achieved = launch_bytes / (per / 1e3) / 1e9
    step_bytes = launch_bytes * (p - 1)
    out = {"metric": METRIC,
           "value": round(step_bytes * its / (rep["time_filter_ms"] / 1e3) / 1e9, 1),
           "unit": "GB/s", "n_gpus": 1, "steps": its, "warmup": warmup,
           "ms_per_step": round(wall * 1e3 / its, 2), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": prec_name, "data": "synthetic",
           "config": {"workload": f"periodic {g}^3 grid pencil, 27-point Q1 stiffness/mass, "
                                  f"{wells} Gaussian wells (mass-weighted), block {b}, "
                                  f"{nw} wanted, degree {p}, {prec_name} residual filter" +
                                  (f", Bloch wave vector {kvec} (complex)" if kvec else ""),
                      "n": n, "block": b, "degree": p, "memory_mode": mode,
                      "lambda_max_estimate": round(lmax, 6),
                      "bounds_estimate_ms": round(bounds_ms, 1),
                      "filter_ms_per_step": round(rep["time_filter_ms"] / its, 2),
                      "rr_ms_per_step": round(rep["time_rr_ms"] / its, 2),
                      "jacobi_sweeps": rep["jacobi_sweeps"],
                      "max_residual_after": rep["max_residual"]},
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                        "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4),
                        "traffic": (TRAFFIC_BLOCH_STEP if kvec else TRAFFIC_ZMARCH).get(
                            (g, b, prec_name)),
                        "traffic_unit": "bytes per launch",
                        "kernel": f"k_zmarch<{prec_name}> residual-filter step "
                                  f"(4 streams x {esize} B per element-step)" +
                                  (" + k_bloch boundary-correction pass" if kvec else ""),
                        "ms_per_launch": round(per, 3)}}
    ctx.close()
    del X
    torch.cuda.synchronize()
    state = {"P": P, "prob": prob, "n": n, "b": b, "nw": nw, "p": p, "kvec": kvec, "prec": prec,
             "Vd": Vd, "opA": opA, "opB": opB, "stream": stream, "lmax": lmax, "esize": esize}
    return out, state


def grid_cpu_baseline(prob, seconds_target=10.0):
    """The oracle's C/OpenMP FP64 residual filter (Algorithm 3, oracle/stencil27.c) on a
    column panel of the grid pencil; the filter is column-independent, so the rate
    per column scales to the block.  Reported in the workload's unit: element-steps
    per second times the BF16 filter's 8 algorithmic bytes per element-step."""
    import numpy as np
    from oracle import cstencil
    n, p, shape = prob.n, prob.degree, prob.shape
    rng = np.random.default_rng(7)
    lam = np.sort(rng.uniform(-4.0, 1.0, 64))
    bounds = (-4.5, 18.5, 1.0)

    def run(k):
        X = rng.standard_normal((n, k))
        R = 1e-3 * rng.standard_normal((n, k))
        t0 = time.perf_counter()
        cstencil.rchfsi_filter(prob.coef_A, prob.coef_B, prob.V, prob.field_mode, shape, None, X,
                               lam[:k], R, p, *bounds)
        return time.perf_counter() - t0

    t1 = run(1)
    k = int(max(1, min(64, seconds_target / max(t1, 1e-3))))
    dt = run(k) if k > 1 else t1
    el_steps = float(n) * k * (p - 1)
    return {"value": round(el_steps * 8.0 / dt / 1e9, 2), "unit": "GB/s",
            "element_steps_per_s": round(el_steps / dt, 1), "cores": cstencil.threads(),
            "kind": "oracle", "cpu_model": host_info()["cpu_model"],
            "sample": f"Algorithm 3 FP64 C/OpenMP grid filter (oracle/stencil27.c), "
                      f"{shape[0]}^3 grid, {k} of {prob.block} columns (the filter is "
                      f"column-independent), degree {p}, {dt:.2f} s; rate in element-steps "
                      f"x 8 B (the BF16 filter's algorithmic bytes per element-step)"}


def bench_grid(args):
    """Grid workload line: timed outer iterations, optionally the time-to-residual runs."""
    import torch

    out, S = grid_steps(args.grid, args.wells, args.prec, args.bloch, args.steps, args.warmup,
                        degree=args.degree if args.degree != 20 else None)
    P, n, b, nw, p, kvec, prec = S["P"], S["n"], S["b"], S["nw"], S["p"], S["kvec"], S["prec"]
    opA, opB, Vd, stream, lmax = S["opA"], S["opB"], S["Vd"], S["stream"], S["lmax"]
    if args.ttr:
        # time to max residual < tau over the wanted pairs, from the same random
        # start (Philox seed 2002): reduced-precision R-ChFSI vs the FP64 baselines;
        # lambda_max = NaN: each solve makes its own Lanczos estimate (included)
        ttr = {}
        runs = [(args.prec + "_rchfsi", P.METHOD_RCHFSI, prec, args.ttr_iters),
                ("fp64_rchfsi", P.METHOD_RCHFSI, P.PREC_FP64, args.ttr_iters),
                ("fp64_chfsi_dinv_identity", P.METHOD_CHFSI, P.PREC_FP64, args.ttr_chfsi_iters)]
        wanted_runs = set(r for r in args.ttr_runs.split(",") if r)
        for name, method, pr, iters in runs:
            if name == "fp64_rchfsi" and prec == P.PREC_FP64:
                continue
            if kvec is not None and method == P.METHOD_CHFSI:
                continue                        # complex contexts run the residual filter only
            if wanted_runs and name not in wanted_runs:
                continue
            pm = P.make_params(nw, b, p, max_iter=iters, tol=1e-8, method=method, filter_prec=pr,
                               seed=2002, init_random=1)
            if args.ttr_escalate > 0 and pr == P.PREC_BF16 and kvec is None:
                pm.stall_iters, pm.escalate = args.ttr_escalate, 1
            md = 0
            torch.cuda.empty_cache()
            free_now = torch.cuda.mem_get_info()[0]
            # the slab-wise Rayleigh-Ritz (memory_mode 1) serves the FP32/BF16
            # residual filters on real grids
            if (kvec is None and pr != P.PREC_FP64 and
                    P.chfsi_workspace_bytes(opA, opB, pm) + n * b * 8 > 0.9 * free_now):
                md = 1
            if args.ttr_memory_mode >= 0 and pr != P.PREC_FP64 and kvec is None:
                md = args.ttr_memory_mode
            pm.memory_mode = md
            need = P.chfsi_workspace_bytes(opA, opB, pm) + n * b * 8 * (2 if kvec else 1)
            if need > 0.9 * free_now and pr == P.PREC_FP64 and kvec is None:
                # the whole FP64 block recurrence does not fit: time its filter by
                # column panels (the filter is column-independent, so the panels'
                # times add up to one full filter pass exactly)
                ttr[name] = fp64_filter_by_panels(P, opA, opB, n, b, nw, p, lmax, stream,
                                                  args.fp64_panel, Vd, need)
                log(f"  {name}: {ttr[name]}")
                continue
            log(f"time-to-residual: {name} (memory_mode {md}) ...")
            c2 = P.chfsi_create(opA, opB, None, pm, stream=stream, keep=(Vd,))
            X2 = P.colmajor_empty(n, b) if kvec is None else P.colmajor_empty_complex(n, b)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st2, ev2, rn2, rep2 = P.chfsi_solve(c2, X2)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t1
            ttr[name] = {"status": "OK" if st2 == P.OK else "ERR_NOCONV", "seconds": round(sec, 2),
                         "iterations": rep2["iterations"], "max_residual": rep2["max_residual"],
                         "filter_ms": round(rep2["time_filter_ms"], 1),
                         "rr_ms": round(rep2["time_rr_ms"], 1), "memory_mode": md,
                         "lambda_max_used": round(rep2["lambda_max_used"], 6),
                         "bounds_ms": round(rep2["time_bounds_ms"], 1),
                         "svqb_events": rep2["svqb_events"], "svqb_dropped": rep2["svqb_dropped"],
                         "escalation_iteration": rep2["escalation_iteration"],
                         "residual_history": [float("%.3g" % v) for v in rep2["history"]]}
            log(f"  {ttr[name]}")
            c2.close()
            del X2
            torch.cuda.synchronize()
        lo = ttr.get(args.prec + "_rchfsi")
        hi = ttr.get("fp64_rchfsi")
        if lo and hi and lo["status"] == "OK" and hi["status"] == "OK":
            ttr["speedup_vs_fp64_rchfsi"] = round(hi["seconds"] / lo["seconds"], 3)
        elif lo and hi and lo["status"] == "OK" and "filter_ms_per_iteration_by_panels" in hi:
            # estimate: the reduced-precision run's iteration count and FP64
            # Rayleigh-Ritz time, with the FP64 filter timed by column panels
            est = (lo["iterations"] * hi["filter_ms_per_iteration_by_panels"] + lo["rr_ms"]) / 1e3
            hi["seconds_estimate"] = round(est, 2)
            ttr["speedup_vs_fp64_rchfsi_estimate"] = round(est / lo["seconds"], 3)
        out["time_to_residual"] = ttr
    if args.calibrate_copy:
        nbytes = args.calibrate_copy * (1 << 20)
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = nbytes
    if not args.no_cpu_baseline and kvec is None:
        log("timing the CPU oracle (C/OpenMP grid filter) ...")
        out["cpu_baseline"] = grid_cpu_baseline(S["prob"])
    print(json.dumps(out), flush=True)


def fp64_filter_by_panels(P, opA, opB, n, b, nw, p, lmax, stream, panel, Vd, need):
    """FP64 residual-filter time of one outer iteration on a block too large for
    device memory, from column panels of `panel` vectors (random Ritz-like
    data; the filter's time does not depend on the values)."""
    import numpy as np
    import torch
    panel = min(panel, b)
    pm = P.make_params(min(nw, panel), panel, p, max_iter=1, tol=0.0,
                       method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP64, lambda_max=lmax,
                       seed=7, init_random=0, profile=1)
    ctx = P.chfsi_create(opA, opB, None, pm, stream=stream, keep=(Vd,))
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    X = torch.randn((panel, n), dtype=torch.float64, device="cuda", generator=g).t()
    R = torch.randn((panel, n), dtype=torch.float64, device="cuda", generator=g).t()
    Y = P.colmajor_empty(n, panel)
    ritz = [float(v) for v in np.linspace(-4.0, 1.0, panel)]
    P.chfsi_filter(ctx, X, ritz, R, Y, -4.5, lmax, 1.0, degree=p)   # warm-up
    torch.cuda.synchronize()
    P.chfsi_filter_kernel_time(ctx)
    t0 = time.perf_counter()
    P.chfsi_filter(ctx, X, ritz, R, Y, -4.5, lmax, 1.0, degree=p)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    kms, launches = P.chfsi_filter_kernel_time(ctx)
    ctx.close()
    del X, R, Y
    torch.cuda.synchronize()
    panels = b / panel
    return {"status": "does not fit in device memory",
            "bytes_needed": int(need),
            "filter_ms_per_iteration_by_panels": round(sec * 1e3 * panels, 1),
            "step_ms_by_panels": round(kms / max(launches, 1), 3),
            "panel_columns": panel, "panels": round(panels, 3)}


def bench_serving(args):
    """Continuous-batching stream: Poisson arrivals, sequences of perturbed dense pencils
    warm-started from the previous step, FP32 residual filter + FP64 Rayleigh-Ritz."""
    import queue
    import threading

    import numpy as np
    import torch

    import paper_2503_22652_amd as P
    import workloads as wl
    from workloads import gpu as wg

    torch.cuda.set_device(0)
    sizes_all = tuple(int(x) for x in args.sizes.split(","))
    arrivals, sizes = wl.serving_schedule(args.requests, args.sequences, 200.0, sizes_all)
    seqs = []
    t_gen = time.perf_counter()
    for sidx in range(args.sequences):
        n = int(sizes[sidx])
        k = int(math.ceil(0.05 * n))
        b = int(math.ceil(1.25 * k / 16) * 16)
        A, B, dinv, lam = wg.dense_problem(n, k, 3000 + sidx)
        # lambda_max = NaN: each request's solve makes the library's Lanczos estimate
        seqs.append({"n": n, "k": k, "b": b, "A": A, "B": B, "dinv": dinv, "lmax": math.nan,
                     "normA": float(lam.abs().max())})
    torch.cuda.synchronize()
    log(f"serving inputs generated in {time.perf_counter() - t_gen:.1f} s")
    srv = P.Server(slots=args.slots)
    done = []
    q = queue.Queue()

    def waiter():
        while True:
            item = q.get()
            if item is None:
                return
            ticket, meta = item
            r = srv.wait(ticket)
            r.update(meta)
            done.append(r)

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.perf_counter()
    for i in range(args.requests):
        sidx, t = i % args.sequences, i // args.sequences
        sq = seqs[sidx]
        if t > 0:
            E = wg.unit_perturbation(sq["n"], 4000 + 8 * sidx + t)
            sq["A"] = (sq["A"] + 1e-3 * sq["normA"] * E).t().contiguous().t()
            del E
        torch.cuda.current_stream().synchronize()
        now = time.perf_counter() - t0
        if now < arrivals[i]:
            time.sleep(arrivals[i] - now)
        req = P.chfsi_request()
        req.A = P.dense_operator(sq["A"])
        req.B = P.dense_operator(sq["B"])
        req.d_inv = sq["dinv"].data_ptr()
        req.params = P.make_params(sq["k"], sq["b"], 20, max_iter=60, tol=1e-8,
                                   method=P.METHOD_RCHFSI, filter_prec=P.PREC_FP32,
                                   lambda_max=sq["lmax"], seed=5000 + i)
        req.seq_id = sidx
        ticket = srv.submit(req, keep=(sq["A"], sq["B"], sq["dinv"]))
        q.put((ticket, {"seq": sidx, "step": t, "n": sq["n"]}))
    q.put(None)
    th.join()
    wall = time.perf_counter() - t0
    srv.close()
    lat = np.array([r["finish_ms"] - r["submit_ms"] for r in done])
    ok = [r for r in done if r["status"] == P.OK]
    its_first = [r["iterations"] for r in done if r["step"] == 0]
    its_warm = [r["iterations"] for r in done if r["step"] > 0]
    out = {"metric": METRIC, "value": round(float(np.percentile(lat, 99)), 2), "unit": "ms (p99 latency)",
           "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f32",
           "config": {"workload": f"serving: {args.requests} dense generalized solves, "
                                  f"{args.sequences} sequences, Poisson 200/s, N in {sizes_all}, "
                                  f"k = 5% N, degree 20, FP32 R-ChFSI, warm start, {args.slots} slots"},
           "p50_ms": round(float(np.percentile(lat, 50)), 2),
           "p99_ms": round(float(np.percentile(lat, 99)), 2),
           "throughput_solves_per_s": round(len(done) / wall, 2),
           "converged": len(ok), "requests": len(done),
           "mean_iterations_cold": round(float(np.mean(its_first)), 2) if its_first else None,
           "mean_iterations_warm": round(float(np.mean(its_warm)), 2) if its_warm else None,
           "max_residual_max": max(r["max_residual"] for r in done)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

"""Benchmark of the reciprocal incoherent-light average on one MI355X.

One step = one inverse-design evaluation of each of B fresh seeded geometries
(B = 8 by default, factored side by side in the same launches): pillar widths
-> permittivity map -> FDFD assembly -> twisted block factorisation ->
reciprocal solve -> Toeplitz/FFT form F = v^dag W v -> adjoint solve ->
dF/deps -> dF/dwidths, all in librecip's HIP kernels, inputs already on the
device.  value = evaluations per second (B per step).

Beside it, on the factors of the last step: the reciprocal average with cached
factors, the 1000-node Gauss-Legendre brute force it replaces (the same
solver over 1000 planewave right-hand sides), the average over 16 outputs under
a non-translation-invariant (dense W) correlated light, a broadband evaluation
(the geometry at 8 wavelengths, factored side by side), a few batched L-BFGS-B
iterations of inverse design, the FP32-factor + FP64-refinement
variant (one geometry, and the B geometries factored side by side), the
factorisation rate (LU TF/s), the live roofline of the dominant
kernel (HIP events on the launching stream), and the FP64 CPU oracle timed on
a bounded sample of the same workload.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import threading
import time
from dataclasses import replace

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "avg-intensity evals/s reciprocal vs 1000-angle brute force; LU TF/s; p99 ms"
FP64_PEAK_TFLOPS = 78.6     # MI355X dense FP64 matrix peak
FP32_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    import workloads as W
    return {"config1": W.config1, "config2": W.config2, "config3": W.config3,
            "config4_large": W.config4_large}[name]()


DESCR = {
    "config1": "concentrator 10x8 wavelengths (240x200 cells), 10 seeded pillars, cone +-10 deg",
    "config2": "concentrator 100 wavelengths wide, focal distance 50 (2040x1080 cells), "
               "100 seeded pillars, cone +-20 deg",
    "config3": "collimator 200x20 wavelengths (4040x440 cells), 200 seeded pillars, "
               "annulus 10-30 deg and mirror",
    "config4_large": "concentrator 100x20 wavelengths (2040x440 cells), 100 seeded pillars, "
                     "cone +-10 deg",
}


# HBM traffic of the dominant kernel, k_gj2_fused<double> (two panels per pass),
# per launch, from two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE) over one
# default step (config2, eight geometries per step), scaled by what the same
# counters read for a 1 GiB copy (python bench.py --calibrate-copy).  Valid only
# for the kernel source it was measured on: reported when factor.hip still has
# this hash.
TRAFFIC = {"config": "config2", "batch": 8,
           "sha256": "8bc93d15c917f139243825beae9a882640172eaccb869caab350322403945947",
           "fetch_bytes": 180047288,     # 87916.1 KiB FETCH_SIZE x 1.99995
           "write_bytes": 156773037}    # 153098.7 KiB WRITE_SIZE x 1.00000


def factor_source_sha256():
    import hashlib
    path = os.path.join(ROOT, "paper_2207_10701_amd", "csrc", "factor.hip")
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def measured_traffic(config, batch):
    """Bytes per launch of k_gj2_fused<double> if measured on this source and workload."""
    t = TRAFFIC
    if t is None or t["config"] != config or t["batch"] != batch:
        return None
    if t["sha256"] != factor_source_sha256():
        return None
    return t["fetch_bytes"] + t["write_bytes"]


def calibrate_copy():
    """A plain 1 GiB device copy, three times: the reference for FETCH_SIZE/WRITE_SIZE."""
    import torch
    n = 1 << 30
    a = torch.ones(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_bytes": n, "copies": 3}), flush=True)


def nominal_lu_flops(p):
    """Dense-equivalent count: a dense complex inverse per block, 8 n^3 flops.  The
    symmetric sweep does about half of it, so rates on this count can exceed the peak."""
    return 8.0 * p.ny ** 3 * p.nx


def method_lu_flops(p):
    """The method's own count: the symmetric inverse of a complex n x n block costs
    4 n^3 flops (n columns, each a rank-1 update of the symmetric half, 8 flops per
    complex multiply-add), n = ny unpadded."""
    return 4.0 * p.ny ** 3 * p.nx


def executed_lu_flops(p):
    """Complex multiply-adds the symmetric tile sweep executes, at 8 flops each: per
    block, nt panels each updating the nt (nt + 1) / 2 packed 32 x 32 tiles with a
    rank-32 complex product (padded rows and whole diagonal tiles included).  The
    matrix cores take three real products per complex one in most of them, so they
    execute fewer real flops than this (mfma_real_pass_flops)."""
    nt = -(-p.ny // 32)
    return 8.0 * 32 ** 3 * nt * (nt * (nt + 1) // 2) * p.nx


def mfma_real_pass_flops(nt, chains):
    """Real flops the matrix cores execute in one two-panel pass of `chains` blocks of
    nt x nt packed tiles: rank-64 updates in three real products per complex one
    (6 flops per complex multiply-add) on the tiles outside columns K, K+1 and the next
    pivot pair; rank-32 four-product updates (8 flops) on column K; the pivot work
    (three rank-64 quadrant updates, Q3_K4, D4' and the K3 row tile of panel K4) in
    three products.  Columns K+1 are copies."""
    tb3 = 32.0 ** 3
    regular = nt * (nt + 1) // 2 - nt - (nt - 1) - 3
    per_chain = regular * 2 * 6 * tb3 + (nt - 1) * 8 * tb3 + (3 * 2 + 3) * 6 * tb3
    return chains * per_chain


def lu_rates(p, seconds, count=1, peak=None):
    peak = FP64_PEAK_TFLOPS if peak is None else peak
    m = count * method_lu_flops(p) / seconds / 1e12
    return {"tflops_method_4n3": round(m, 3),
            "frac_peak_method": round(m / peak, 4),
            "tflops_executed": round(count * executed_lu_flops(p) / seconds / 1e12, 3),
            "tflops_dense_equiv_8n3": round(count * nominal_lu_flops(p) / seconds / 1e12, 3)}


def host_description():
    """nproc, CPU model and the BLAS / OpenMP thread settings of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    env = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS",
                                          "MKL_NUM_THREADS")}
    return {"nproc": os.cpu_count(), "cpu_model": model, "env": env}


def cpu_baseline(p):
    """FP64 oracle on the benchmark workload itself: one geometry of the step
    (SuperLU factor + reciprocal F by the direct Toeplitz double sum + adjoint
    gradient), BLAS limited to one thread (SuperLU is sequential anyway)."""
    import workloads as W
    from oracle import average as ora
    try:
        from threadpoolctl import threadpool_limits
    except Exception:   # pragma: no cover
        threadpool_limits = None
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    t0 = time.perf_counter()
    s = ora.setup(p)
    g = ora.adjoint(s)
    t = time.perf_counter() - t0
    del s
    if ctx is not None and hasattr(ctx, "unregister"):
        ctx.unregister()
    return {"value": 1.0 / t, "unit": "evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one geometry of the benchmark workload itself ({p.nx}x{p.ny} cells, "
                      f"the first seeded widths of the step): SuperLU/COLAMD factor + reciprocal F "
                      f"(direct O(M^2) Toeplitz sum) + adjoint gradient, {t:.1f} s on one thread; "
                      f"sparse LU with a fill-reducing ordering is a different, asymptotically "
                      f"cheaper algorithm than block elimination",
            "sample_seconds": round(t, 2), "sample_F": g.F, "host": host_description()}


def serving(args):
    """The serving mix as stated: a seeded Poisson stream at 200 requests/s of
    concentrator and collimator evaluations, widths 20-300 and depths 10-60
    wavelengths (every geometry fresh), 20% with an adjoint gradient, served
    with continuous batching (the factorisation engine: every geometry in flight
    advances in shared launches, new ones join between rounds; evaluations on
    four streams beside it) and admission by factor memory, against the same
    stream served one request at a time (plain FP64, factored alone, nothing
    cached).  Then two smaller mixes where the factor cache and shared
    multi-RHS sweeps matter."""
    import torch

    import workloads as W
    from paper_2207_10701_amd.serve import GpuExecutor, Server, serve_sequential, summarize
    reqs = W.serving_stream(args.serve_requests, rate=200.0, seed=5001, scale=args.serve_scale,
                            adjoint_frac=0.2)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    free, total = torch.cuda.mem_get_info()
    budget = int(free - (24 << 30))
    ex = GpuExecutor()
    # warm the kernels once
    warm = Server(ex, hbm_budget=budget, cache=False)
    warm.run(reqs[:1], realtime=False)
    warm.close()
    torch.cuda.synchronize()
    # two factorisation engines on two streams, up to 16 geometries in flight
    conc = Server(ex, factor_slots=16, eval_slots=4, hbm_budget=budget, cache=True, engines=2)
    res = conc.run(reqs, realtime=True)
    conc.close()
    s_con = summarize(res)
    log(f"serving: engine {s_con}, occupancy {conc.engine_occupancy():.2f}")
    errors = sorted({r.error for r in res if r.error})[:3]
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # the same stream with the largest factorisations admitted first
    lpt = Server(ex, factor_slots=16, eval_slots=4, hbm_budget=budget, cache=True,
                 order="largest_first", engines=2)
    res_l = lpt.run(reqs, realtime=True)
    lpt.close()
    s_lpt = summarize(res_l)
    log(f"serving: engine, largest first {s_lpt}, occupancy {lpt.engine_occupancy():.2f}")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # the same stream on complex-FP32 factors with FP64 refinement (half the
    # factor memory per geometry, twice the matrix-core rate)
    import paper_2207_10701_amd as rcp
    ex32 = GpuExecutor(precision=rcp.RCP_FP32_REFINED)
    f32 = Server(ex32, factor_slots=16, eval_slots=4, hbm_budget=budget, cache=True, engines=2)
    res_32 = f32.run(reqs, realtime=True)
    f32.close()
    s_32 = summarize(res_32)
    ref = {r.rid: r.F for r in res if r.F is not None}
    dF = [abs(r.F - ref[r.rid]) / abs(ref[r.rid]) for r in res_32
          if r.F is not None and r.rid in ref and ref[r.rid] != 0]
    log(f"serving: engine, FP32 refined {s_32}, occupancy {f32.engine_occupancy():.2f}")
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    # one engine (up to 8 geometries in flight), FP64 and FP32 refined
    one = {}
    for name, exe in (("fp64", ex), ("fp32_refined", ex32)):
        srv2 = Server(exe, factor_slots=8, eval_slots=4, hbm_budget=budget, cache=True, engines=1)
        res2 = srv2.run(reqs, realtime=True)
        srv2.close()
        s2 = summarize(res2)
        one[name] = {"p50_ms": round(s2["p50_ms"], 2), "p99_ms": round(s2["p99_ms"], 2),
                     "evals_per_s": round(s2["evals_per_s"], 3), "makespan_s": round(s2["makespan_s"], 3),
                     "max_geometries_factoring": srv2.max_factoring,
                     "engine_mean_geometries": round(srv2.engine_occupancy(), 2), "failed": s2["failed"]}
        log(f"serving: one engine, {name} {s2}, occupancy {srv2.engine_occupancy():.2f}")
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    seq = serve_sequential(ex, reqs, realtime=True)
    s_seq = summarize(seq)
    log(f"serving: sequential {s_seq}")
    work = sum(4.0 * q.problem.ny ** 3 * q.problem.nx for q in reqs)
    out = {"stream": f"{len(reqs)} requests, Poisson 200/s (seed 5001, geometries seed 5002), "
                     f"widths 20-300 and depths 10-60 wavelengths x{args.serve_scale}, "
                     f"50/50 concentrator/collimator, cone or annulus, 20% adjoint",
           "requests": len(reqs), "rate_per_s": 200.0, "scale": args.serve_scale,
           "factor_work_tflop_method": round(work / 1e12, 1),
           "factor_slots": 16, "engines": 2, "eval_slots": 4, "hbm_budget_gb": round(budget / 2 ** 30, 1),
           "p50_ms": round(s_con["p50_ms"], 2), "p99_ms": round(s_con["p99_ms"], 2),
           "evals_per_s": round(s_con["evals_per_s"], 3), "makespan_s": round(s_con["makespan_s"], 3),
           "factor_tflops_method": round(work / s_con["makespan_s"] / 1e12, 2)
           if s_con["makespan_s"] > 0 else None,
           "max_geometries_factoring": conc.max_factoring, "max_evaluations": conc.max_inflight,
           "engine_mean_geometries": round(conc.engine_occupancy(), 2),
           "engine_mean_geometries_note": "per engine, time-weighted while it runs",
           "admission": "arrival order (first come, first served for memory and engine slots)",
           "largest_first": {"p50_ms": round(s_lpt["p50_ms"], 2), "p99_ms": round(s_lpt["p99_ms"], 2),
                             "evals_per_s": round(s_lpt["evals_per_s"], 3),
                             "makespan_s": round(s_lpt["makespan_s"], 3),
                             "engine_mean_geometries": round(lpt.engine_occupancy(), 2),
                             "failed": s_lpt["failed"]},
           "fp32_refined": {"p50_ms": round(s_32["p50_ms"], 2), "p99_ms": round(s_32["p99_ms"], 2),
                            "evals_per_s": round(s_32["evals_per_s"], 3),
                            "makespan_s": round(s_32["makespan_s"], 3),
                            "engine_mean_geometries": round(f32.engine_occupancy(), 2),
                            "max_rel_diff_F_vs_fp64": max(dF) if dF else None,
                            "failed": s_32["failed"]},
           "one_engine": {"note": "one factorisation engine, up to 8 geometries in flight", **one},
           "peak_ledger_gb": round(conc.peak_bytes / 2 ** 30, 2),
           "failed": s_con["failed"], "errors": errors,
           "latency_note": "from arrival to result; the stream offers far more work than one GPU "
                           "serves, so latency is queue-dominated",
           "sequential_fp64": {"p50_ms": round(s_seq["p50_ms"], 2),
                               "p99_ms": round(s_seq["p99_ms"], 2),
                               "evals_per_s": round(s_seq["evals_per_s"], 3),
                               "makespan_s": round(s_seq["makespan_s"], 3),
                               "failed": s_seq["failed"]},
           "speedup_vs_sequential": round(s_con["evals_per_s"] / s_seq["evals_per_s"], 3)
           if s_seq["evals_per_s"] > 0 else None}
    if args.serve_extras:
        # the same kind of stream over a seeded pool of 16 geometries at a quarter
        # of the size: cached factors serve repeated geometries
        preqs = W.serving_stream(24, rate=200.0, seed=5001, scale=0.25, adjoint_frac=0.2,
                                 geometry_pool=16)
        pool = Server(ex, hbm_budget=budget, cache=True)
        pres = pool.run(preqs, realtime=True)
        pool.close()
        s_pool = summarize(pres)
        out["geometry_pool_16_scale_0.25"] = {
            "requests": len(preqs), "p50_ms": round(s_pool["p50_ms"], 2),
            "p99_ms": round(s_pool["p99_ms"], 2), "evals_per_s": round(s_pool["evals_per_s"], 3),
            "cache_hits": sum(1 for r in pres if r.cache_hit),
            "shared_sweep_requests": sum(1 for r in pres if r.group > 1),
            "failed": s_pool["failed"]}
        # a backlog: 64 plain requests over 4 geometries, all waiting at the start;
        # requests on cached factors share one multi-RHS sweep (group 16) or not (1)
        breqs = W.serving_stream(64, rate=200.0, seed=5004, scale=0.25, adjoint_frac=0.0,
                                 geometry_pool=4)
        backlog = {}
        for g in (16, 1):
            srv = Server(ex, hbm_budget=budget, cache=True, group=g)
            bres = srv.run(breqs, realtime=False)
            srv.close()
            sb = summarize(bres)
            backlog[f"group_{g}"] = {"evals_per_s": round(sb["evals_per_s"], 3),
                                     "p99_ms": round(sb["p99_ms"], 2), "failed": sb["failed"],
                                     "shared_sweep_requests": sum(1 for r in bres if r.group > 1)}
        out["backlog_64_on_4_geometries_scale_0.25"] = backlog
    return out


def threed_extra(args):
    """The 3D vector problem (Sec. "Concluding remarks") at a size where the
    blocks fill the GPU: 4 x 4 wavelengths of pillars, 2.5 wavelengths deep, h =
    lambda / 8 (48 x 48 x 36 cells, n = 3 ny nz = 5184 unknowns per x-slice, 48
    slices).  Times the factorisation (one geometry through the engine), the
    reciprocal average of a focal spot (three solves) and the forward average
    over a rule of 4 x 16 directions, both polarisations (128 solves)."""
    import torch

    import workloads as W
    from paper_2207_10701_amd import maxwell3d as M
    p3 = W.metasurface3d("bench3d", 4, 2.5, 3001, npml=8, focus_height=0.5, c_deg=20.0)
    n = 3 * p3.ny * p3.nz
    eps = M.eps_from_pillars(p3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = M.Factors3D(p3, eps)
    torch.cuda.synchronize()
    t_f = time.perf_counter() - t0
    th, az, wt = W.cone_directions3d(p3, 4, 16)
    dirs = M.directions(th, az, wt)
    F = M.reciprocal_average(fac, dirs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        F = M.reciprocal_average(fac, dirs)
    torch.cuda.synchronize()
    t_rec = (time.perf_counter() - t0) / 3
    t0 = time.perf_counter()
    Fb = M.brute_force_average(fac, dirs)
    torch.cuda.synchronize()
    t_bf = time.perf_counter() - t0
    work = 4.0 * n ** 3 * p3.nx
    out = {"grid": [p3.nx, p3.ny, p3.nz], "unknowns_per_slice": n, "slices": p3.nx,
           "factor_gb": round(fac.nbytes / 2 ** 30, 2), "factor_seconds": round(t_f, 4),
           "factor_tflops_method_4n3": round(work / t_f / 1e12, 2),
           "frac_peak_method": round(work / t_f / 1e12 / FP64_PEAK_TFLOPS, 4),
           "reciprocal_ms": round(t_rec * 1e3, 3), "reciprocal_solves": 3,
           "directions": len(th), "brute_force_solves": 2 * len(th),
           "brute_force_ms": round(t_bf * 1e3, 3), "speedup_cached": round(t_bf / t_rec, 2),
           "F": F.item(), "rel_diff_brute_force": abs(Fb.item() - F.item()) / abs(F.item())}
    fac.release()
    return out


def dense_extra(args, rcp, W, p, fac, t_rec, stream):
    """Any correlation W and many outputs on cached factors.

    Light: a finite ensemble of planewaves at evenly spaced angles of the cone
    with Gaussian-correlated amplitudes (correlation width 1 deg, phase tilt):
    not translation invariant, so W is dense.  Outputs: focal spots on the focal
    row plus planewave output modes.  Times the ensemble W build (two complex
    matrix products), the K-output average (one multi-RHS reciprocal sweep + the
    dense form W V) and its gradient, against K single-output reciprocal solves.
    """
    import torch
    dev = fac.buf.device
    K, N = args.dense_outputs, args.dense_angles
    outs = W.output_set(p, K - K // 4, K // 4, seed=3700)
    th = W.ensemble_angles(p, N)
    Ca = W.gaussian_correlated_amplitudes(th, sigma_deg=1.0, tilt=5.0)
    th_d = torch.from_numpy(th).to(dev)
    C_d = torch.from_numpy(Ca).to(dev)
    M = p.m_aperture
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    Wm = rcp.correlation_matrix(p, th_d, C_d)           # warm
    need = int(rcp.lib.rcp_dense_work_bytes(fac.handle, K, M))
    work = torch.empty(need, dtype=torch.uint8, device=dev)
    F = rcp.reciprocal_average_dense(fac, outs, Wm, work=work)
    torch.cuda.synchronize()
    reps = 5
    a.record(stream)
    for _ in range(reps):
        Wm = rcp.correlation_matrix(p, th_d, C_d)
    b.record(stream)
    torch.cuda.synchronize()
    t_w = a.elapsed_time(b) * 1e-3 / reps
    w_flops = 8.0 * N * N * M + 8.0 * M * M * N
    rcp.kernel_timing_start(1)
    a.record(stream)
    for _ in range(reps):
        F = rcp.reciprocal_average_dense(fac, outs, Wm, work=work)
    b.record(stream)
    torch.cuda.synchronize()
    kt = rcp.kernel_timing_stop()["dense_zgemm"]
    t_d = a.elapsed_time(b) * 1e-3 / reps
    a.record(stream)
    Fa, g = rcp.adjoint_grad_dense(fac, outs, Wm, work=work)
    b.record(stream)
    torch.cuda.synchronize()
    t_g = a.elapsed_time(b) * 1e-3
    form_us = 1e3 * kt["ms"] / max(kt["samples"], 1)
    form_flops = 8.0 * M * M * K
    form_bytes = 16.0 * M * M + 2 * 16.0 * M * K
    return {"outputs": K, "angles": N, "line_cells": M,
            "W_build_ms": round(1e3 * t_w, 3),
            "W_build_tflops": round(w_flops / t_w / 1e12, 3),
            "average_ms": round(1e3 * t_d, 3), "adjoint_ms": round(1e3 * t_g, 3),
            "single_output_reciprocal_ms_x_K": round(1e3 * t_rec * K, 3),
            "speedup_vs_K_single_solves": round(t_rec * K / t_d, 2),
            "forward_solves_replaced": N * K,
            "form_zgemm_us": round(form_us, 3),
            "form_zgemm_tflops": round(form_flops / (form_us * 1e-6) / 1e12, 3),
            "form_zgemm_gbs": round(form_bytes / (form_us * 1e-6) / 1e9, 1),
            "F_total": F[-1].item(), "F_total_adjoint": Fa[-1].item()}


def broadband_extra(args, rcp, W, p, widths, bufs, stream):
    """One broadband evaluation: the geometry factored at n wavelengths of a flat
    spectral rule over [0.9, 1.1] side by side, then the weighted average and its
    gradient (the batched reciprocal and adjoint solves of all wavelengths)."""
    import torch
    from dataclasses import replace
    n = args.broadband
    lams, wts = W.spectral_rule(n, 0.9, 1.1)
    probs = [replace(p, wavelength=float(lam)) for lam in lams]
    dev = bufs[0].device
    eps = rcp.eps_from_widths(p, widths, device=dev)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    facs = rcp.factor_batch(probs, [eps] * n, rcp.RCP_FP64, buffers=bufs[:n])
    F, g = rcp.broadband_grad(facs, wts, probs)
    b.record(stream)
    torch.cuda.synchronize()
    t = a.elapsed_time(b) * 1e-3
    del facs
    return {"wavelengths": n, "band": [0.9, 1.1], "seconds": round(t, 4),
            "evals_per_s": round(1.0 / t, 4), "F_broadband": F[-1].item(),
            "F_min": F[:-1].min().item(), "F_max": F[:-1].max().item()}


def design_extra(args, W, p, B, bufs):
    """A few L-BFGS-B iterations of B seeded designs of the workload, every round
    of evaluations one batched factorisation + batched adjoint."""
    import torch
    from dataclasses import replace
    from paper_2207_10701_amd.design import gpu_batch_fn, maximize
    probs = [replace(p, name=f"design{k}", widths=W.seeded_widths(len(p.widths), 9000 + k))
             for k in range(B)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, lock = maximize(probs, gpu_batch_fn(buffers=bufs), iters=args.design_iters)
    t = time.perf_counter() - t0
    return {"designs": B, "iters": args.design_iters, "seconds": round(t, 3),
            "rounds": lock.rounds, "evaluations": lock.evaluations,
            "evaluations_per_s": round(lock.evaluations / t, 3),
            "gain_min": round(min(r.F / r.F0 for r in res), 3),
            "gain_max": round(max(r.F / r.F0 for r in res), 3)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="config2", choices=sorted(DESCR))
    ap.add_argument("--bf-angles", type=int, default=1000)
    ap.add_argument("--bf-chunk", type=int, default=1000)
    # each timed launch is bracketed by two event packets, which hold the next
    # launch back by a few microseconds: sample sparsely
    ap.add_argument("--timing-every", type=int, default=32)
    ap.add_argument("--no-extras", action="store_true", help="time the step only")
    ap.add_argument("--factor-batch-only", choices=["fp64", "fp32"], default=None,
                    help="only factor one batch of the workload's geometries (for profiles)")
    ap.add_argument("--no-threed", dest="threed", action="store_false",
                    help="skip the 3D vector problem extra")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=64,
                    help="requests of the serving stream (0 = skip)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="width/depth scale of the serving stream (1 = widths 20-300, depths 10-60)")
    ap.add_argument("--no-serve-extras", dest="serve_extras", action="store_false",
                    help="skip the geometry-pool and backlog serving runs")
    ap.add_argument("--batch", type=int, default=8,
                    help="geometries factored side by side per step (1-8)")
    ap.add_argument("--dense-outputs", type=int, default=16,
                    help="outputs of the dense-correlation extra (0 = skip)")
    ap.add_argument("--design-iters", type=int, default=2,
                    help="L-BFGS-B iterations of the inverse-design extra (0 = skip)")
    ap.add_argument("--broadband", type=int, default=8,
                    help="wavelengths of the broadband extra (0 = skip; at most --batch)")
    ap.add_argument("--dense-angles", type=int, default=1000,
                    help="planewaves in the correlated ensemble of the dense extra")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (reference for the HBM counters)")
    args = ap.parse_args()
    if args.calibrate_copy:
        calibrate_copy()
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; the reciprocal solve of one "
                                   "geometry is not sharded (N must be 1)"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2207_10701_amd as rcp
    import workloads as W

    p = workload(args.config)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.factor_batch_only:
        # one batch of the step's geometries factored alone (a warm-up, then
        # timed), for profiling the factorisation kernels of one precision
        prec = rcp.RCP_FP64 if args.factor_batch_only == "fp64" else rcp.RCP_FP32_REFINED
        # up to 16 with FP32 factors (two groups on two streams); FP64 factors of
        # more than eight config-2 geometries exceed the HBM
        B = max(1, min(16 if prec == rcp.RCP_FP32_REFINED else 8, args.batch))
        eps_b = [rcp.eps_from_widths(p, torch.tensor(W.seeded_widths(len(p.pillar_centers), 1002 + 97 * k),
                                                     dtype=torch.float64, device=dev), device=dev)
                 for k in range(B)]
        nbytes = rcp.factor_bytes(p, prec)
        bufs = [torch.empty(nbytes, dtype=torch.uint8, device=dev) for _ in range(B)]
        rcp.factor_batch([p] * B, eps_b, prec, buffers=bufs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rcp.factor_batch([p] * B, eps_b, prec, buffers=bufs)
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        peak = FP64_PEAK_TFLOPS if prec == rcp.RCP_FP64 else FP32_PEAK_TFLOPS
        print(json.dumps({"factor_batch_only": args.factor_batch_only, "geometries": B,
                          "seconds": round(t, 5), **lu_rates(p, t, B, peak)}), flush=True)
        return
    log(f"bench: {p.name} {p.nx}x{p.ny}, steps={args.steps} warmup={args.warmup}")

    # inputs resident in HBM before timing: B seeded geometries per step
    B = max(1, min(8, args.batch))
    nsteps = args.warmup + args.steps
    widths = [torch.tensor(W.seeded_widths(len(p.pillar_centers), 1002 + 97 * k), dtype=torch.float64,
                           device=dev) for k in range(nsteps * B)]
    # two sets of factor buffers when they fit in 200 GiB (B = 4 on config 2:
    # 8 x ~20 GB): the adjoint evaluations of step k then run while step k+1 is
    # factored; with one set (B = 8) they finish before the next factorisation
    fbytes = rcp.factor_bytes(p, rcp.RCP_FP64)
    nsets = 2 if B > 1 and 2 * B * fbytes <= (200 << 30) else 1
    bufsets = [[torch.empty(fbytes, dtype=torch.uint8, device=dev) for _ in range(B)]
               for _ in range(nsets)]
    bufs = bufsets[0]
    buf = bufs[0]

    # the B adjoint evaluations of a step: one batched call (their solves share
    # kernel launches) on a side stream, issued from a worker thread so that it
    # can overlap the next factorisation (ctypes releases the GIL)
    side = torch.cuda.Stream(device=dev) if B > 1 else None

    def adjoint_on(facs, ws, out):
        with torch.cuda.stream(side):
            Fb, grads = rcp.adjoint_grad_batch(facs, [p] * B, stream=side)
            gws = [rcp.width_grad(p, g, w, stream=side) for g, w in zip(grads, ws)]
            done = torch.cuda.Event(enable_timing=True)
            done.record(side)
            out[:] = [(Fb[j], gws[j], done) for j in range(B)]

    def factor_step(k):
        """ε maps and factorisation of step k (returns once the factors are complete)."""
        ws = widths[k * B:(k + 1) * B]
        eps = [rcp.eps_from_widths(p, w, device=dev) for w in ws]
        if B == 1:
            return [rcp.Factors(p, eps[0], rcp.RCP_FP64, buffer=bufs[0])], ws
        return rcp.factor_batch([p] * B, eps, rcp.RCP_FP64, buffers=bufsets[k % nsets]), ws

    def start_adjoints(facs, ws):
        if B == 1:
            F, g = rcp.adjoint_grad(facs[0], p)
            gw = rcp.width_grad(p, g, ws[0])
            done = torch.cuda.Event(enable_timing=True)
            done.record(stream)
            return None, [(F, gw, done)], facs
        side.wait_stream(stream)
        out = []
        threads = [threading.Thread(target=adjoint_on, args=(facs, ws, out))]
        threads[0].start()
        return threads, out, facs

    def finish_adjoints(pending):
        threads, out, facs = pending
        for t in threads or []:
            t.join()
        if side is not None:
            stream.wait_stream(side)
        if len(out) != len(facs):
            raise RuntimeError("an adjoint evaluation failed")
        return facs[-1], out

    def run(first, count, starts=None):
        """Steps first .. first+count-1, adjoints of step k overlapping factorisation k+1."""
        results, pending = [], None
        if count == 0:
            return results
        for k in range(first, first + count):
            if pending is not None and nsets == 1:   # its factors are about to be overwritten
                results.append(finish_adjoints(pending))
                pending = None
            # a step's latency clock starts once the previous step's adjoints
            # no longer hold its factor buffers
            if starts is not None:
                starts.append(torch.cuda.Event(enable_timing=True))
                starts[-1].record(stream)
            facs, ws = factor_step(k)
            if pending is not None:
                results.append(finish_adjoints(pending))
            pending = start_adjoints(facs, ws)
        results.append(finish_adjoints(pending))
        return results

    for fac, out in run(0, args.warmup):
        torch.cuda.synchronize()
        log(f"warmup: F={out[-1][0].item():.6e}")

    starts = []
    rcp.kernel_timing_start(args.timing_every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = run(args.warmup, args.steps, starts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kstats = rcp.kernel_timing_stop()
    fac = results[-1][0]
    Fs = [r[1][-1][0] for r in results]
    # latency of a step: from the start of its factorisation to its last adjoint result
    lat = sorted(max(a.elapsed_time(o[2]) for o in r[1]) for a, r in zip(starts, results))
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    log(f"timed: {ms_per_step:.1f} ms/step, F={[round(f.item(), 8) for f in Fs]}")
    p50 = float(np.percentile(lat, 50))
    p99 = float(np.percentile(lat, 99))

    upd = kstats["gj_update"]
    # the kernel timer counts executed flops (two panels x every packed tile of
    # each chain's block); the roofline takes the method's count for the same
    # work: 64 columns of a 4 n^3 symmetric inverse, 4 n^2 flops per column
    nt = -(-p.ny // 32)
    method_per_exec = (64 * 4.0 * p.ny ** 2) / (2 * (nt * (nt + 1) // 2) * 8.0 * 32 ** 3)
    achieved = method_per_exec * upd["work"] / (upd["ms"] * 1e-3) / 1e12 if upd["ms"] > 0 else 0.0
    roofline = {"bound": "mfma", "kernel": "k_gj2_fused<double>", "achieved": round(achieved, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                "traffic": measured_traffic(args.config, B),
                "avg_launch_us": round(1e3 * upd["ms"] / max(upd["samples"], 1), 3),
                "flops_per_launch": method_per_exec * upd["work"] / max(upd["samples"], 1),
                "flop_count": "method: 64 columns x 4 ny^2 per chain (16 chains), 8 flops per "
                              "complex multiply-add; padded rows and whole diagonal tiles not counted"}
    if upd["ms"] > 0 and upd["samples"]:
        # what the matrix cores execute: three real products per complex one
        mfma = mfma_real_pass_flops(nt, 2 * B)
        mfma_rate = mfma * upd["samples"] / (upd["ms"] * 1e-3) / 1e12
        roofline["mfma_real_flops_per_launch"] = mfma
        roofline["mfma_real_tflops"] = round(mfma_rate, 3)
        roofline["mfma_real_frac"] = round(mfma_rate / FP64_PEAK_TFLOPS, 4)
    kernels = {}
    for name, st in kstats.items():
        if st["samples"]:
            per = st["ms"] / st["samples"]
            rate = st["work"] / (st["ms"] * 1e-3) if st["ms"] > 0 else 0.0
            kernels[name] = {"launches": st["launches"], "avg_us": round(1e3 * per, 3),
                             "rate": round(rate / (1e9 if "gemv" in name or name == "schur" else 1e12), 3),
                             "rate_unit": "GB/s" if ("gemv" in name or name == "schur") else "TFLOP/s"}

    out = {"metric": METRIC, "value": round(B * args.steps / wall, 5), "unit": "evals/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{p.name}: {DESCR[p.name]}", "grid": [p.nx, p.ny],
                      "step": "eps map + assemble + factor (B side by side) + reciprocal F + "
                              "adjoint dF/dwidths (B batched; overlapping the next step's "
                              "factorisation when two factor sets fit)",
                      "geometries_per_step": B,
                      "precision": "complex FP64"},
           "step_latency_ms": {"p50": round(p50, 3), "p99": round(p99, 3),
                               "definition": "start of a step's factorisation to its last "
                                             "adjoint result"},
           "F": Fs[-1].item(), "roofline": roofline, "kernels": kernels}

    if not args.no_extras:
        # factorisation alone
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        del fac
        eps = rcp.eps_from_widths(p, widths[-1], device=dev)
        a.record(stream)
        fac = rcp.Factors(p, eps, rcp.RCP_FP64, buffer=buf)
        b.record(stream)
        torch.cuda.synchronize()
        t_fac = a.elapsed_time(b) * 1e-3
        out["lu_single"] = {"seconds": round(t_fac, 5), **lu_rates(p, t_fac)}
        if B > 1:   # the same B geometries factored side by side, as in the step
            eps_b = [rcp.eps_from_widths(p, w, device=dev) for w in widths[-B:]]
            del fac
            torch.cuda.synchronize()
            a.record(stream)
            facs_b = rcp.factor_batch([p] * B, eps_b, rcp.RCP_FP64, buffers=bufs)
            b.record(stream)
            torch.cuda.synchronize()
            t_b = a.elapsed_time(b) * 1e-3
            out["lu_batch"] = {"geometries": B, "seconds": round(t_b, 5), **lu_rates(p, t_b, B)}
            log(f"batched factor x{B}: {t_b * 1e3:.1f} ms "
                f"({out['lu_batch']['tflops_method_4n3']} TF/s on the method's count)")
            fac = facs_b[-1]      # geometry widths[-1] again, now in bufs[-1]
            del facs_b
            # the same geometries through the factorisation engine (the launches
            # serving shares between geometries of any size), then one alone
            eng = rcp.FactorEngine(rcp.RCP_FP64, stream=stream)
            del fac
            torch.cuda.synchronize()
            a.record(stream)
            efacs = [eng.add(p, e, buffer=bb) for e, bb in zip(eps_b, bufs)]
            eng.run()
            b.record(stream)
            torch.cuda.synchronize()
            t_e = a.elapsed_time(b) * 1e-3
            F_e = rcp.reciprocal_average(efacs[-1], p).item()
            del efacs
            torch.cuda.synchronize()
            a.record(stream)
            efac = eng.add(p, eps_b[-1], buffer=bufs[0])
            eng.run()
            b.record(stream)
            torch.cuda.synchronize()
            t_e1 = a.elapsed_time(b) * 1e-3
            eng.close()
            out["lu_engine"] = {"batch": {"geometries": B, "seconds": round(t_e, 5),
                                          **lu_rates(p, t_e, B)},
                                "single": {"seconds": round(t_e1, 5), **lu_rates(p, t_e1)},
                                "F_last": F_e}
            log(f"engine x{B}: {t_e * 1e3:.1f} ms, alone {t_e1 * 1e3:.1f} ms")
            del efac
            facs_b = rcp.factor_batch([p] * B, eps_b, rcp.RCP_FP64, buffers=bufs)
            fac = facs_b[-1]
            del facs_b
        # reciprocal average on cached factors
        reps = 10
        Fr = rcp.reciprocal_average(fac, p)
        torch.cuda.synchronize()
        a.record(stream)
        for _ in range(reps):
            Fr = rcp.reciprocal_average(fac, p, out=Fr)
        b.record(stream)
        torch.cuda.synchronize()
        t_rec = a.elapsed_time(b) * 1e-3 / reps
        out["reciprocal_cached_ms"] = round(1e3 * t_rec, 4)
        log(f"factor {t_fac * 1e3:.1f} ms ({out['lu_single']['tflops_method_4n3']} TF/s method), "
            f"reciprocal cached {t_rec * 1e3:.3f} ms, F={Fr.item():.10e}")
        # the brute force it replaces, same factors
        if p.light in (W.CONE, W.ANNULUS) and args.bf_angles > 0:
            chunk = min(args.bf_chunk, args.bf_angles)
            # once untimed: the block-product library loads its kernels on first use
            rcp.brute_force_average(fac, args.bf_angles, p, rhs_chunk=chunk)
            torch.cuda.synchronize()
            a.record(stream)
            Fb = rcp.brute_force_average(fac, args.bf_angles, p, rhs_chunk=chunk)
            b.record(stream)
            torch.cuda.synchronize()
            t_bf = a.elapsed_time(b) * 1e-3
            rel = abs(Fb.item() - Fr.item()) / abs(Fr.item())
            bf_flops = 16.0 * p.ny ** 2 * p.nx * args.bf_angles
            out["brute_force"] = {
                "angles": args.bf_angles, "rhs_chunk": chunk, "seconds": round(t_bf, 4),
                "evals_per_s_cached": round(1.0 / t_bf, 4),
                "evals_per_s_end_to_end": round(1.0 / (t_bf + t_fac), 4),
                "F": Fb.item(), "rel_diff_vs_reciprocal": rel,
                "gemm_tflops": round(bf_flops / t_bf / 1e12, 3)}
            out["speedup"] = {"solve_count": args.bf_angles,
                              "cached_factors": round(t_bf / t_rec, 2),
                              "end_to_end": round((t_bf + t_fac) / (t_rec + t_fac), 3)}
            log(f"brute force {args.bf_angles} angles: {t_bf:.3f} s, F={Fb.item():.10e}, "
                f"rel diff {rel:.2e}")
            # Sec. "Brute-force quadrature": the Gauss-Legendre rule against the
            # reciprocal F on the same factors as the node count grows
            sweep = []
            for n in (16, 32, 64, 128, 256, 512, 1024):
                torch.cuda.synchronize()
                a.record(stream)
                Fn = rcp.brute_force_average(fac, n, p, rhs_chunk=min(n, 1024)).item()
                b.record(stream)
                torch.cuda.synchronize()
                sweep.append({"nodes": n, "rel_err_vs_reciprocal": abs(Fn - Fr.item()) / Fr.item(),
                              "seconds": round(a.elapsed_time(b) * 1e-3, 4)})
            out["gl_node_sweep"] = {"note": "F_bf(N) of the +-20 deg cone on the config-2 factors "
                                            "against the reciprocal F; resolved once N exceeds "
                                            "about K c L / 2 = 164",
                                    "points": sweep}
            log(f"GL sweep: {[(q['nodes'], '%.1e' % q['rel_err_vs_reciprocal']) for q in sweep]}")
        # any correlation W and many outputs on the same factors
        if args.dense_outputs > 0:
            out["dense_correlation"] = dense_extra(args, rcp, W, p, fac, t_rec, stream)
            log(f"dense: {out['dense_correlation']}")
        # FP32 factors + FP64 refinement, error vs FP64
        del fac
        buf32 = torch.empty(rcp.factor_bytes(p, rcp.RCP_FP32_REFINED), dtype=torch.uint8,
                            device=dev)
        torch.cuda.synchronize()
        a.record(stream)
        f32 = rcp.Factors(p, eps, rcp.RCP_FP32_REFINED, buffer=buf32)
        b.record(stream)
        F32, z32 = rcp.reciprocal_average(f32, p, want_z=True)
        torch.cuda.synchronize()
        t_f32 = a.elapsed_time(b) * 1e-3
        it, res = f32.last_solve_stats()
        t_b32 = None
        if B > 1:   # the step's B geometries with FP32 factors, side by side
            eps_b = [rcp.eps_from_widths(p, w, device=dev) for w in widths[-B:]]
            torch.cuda.synchronize()
            a.record(stream)
            facs32 = rcp.factor_batch([p] * B, eps_b, rcp.RCP_FP32_REFINED, buffers=bufs)
            b.record(stream)
            torch.cuda.synchronize()
            t_b32 = a.elapsed_time(b) * 1e-3
            del facs32, eps_b
        t_b32x2 = None
        if B == 8:   # sixteen geometries with FP32 factors (half the bytes): two groups of eight
            # on two streams of the library, the FP64 step's buffers holding eight of them
            eps_16 = [rcp.eps_from_widths(p, torch.tensor(W.seeded_widths(len(p.pillar_centers), 1002 + 97 * k),
                                                          dtype=torch.float64, device=dev), device=dev)
                      for k in range(16)]
            more = [torch.empty(rcp.factor_bytes(p, rcp.RCP_FP32_REFINED), dtype=torch.uint8, device=dev)
                    for _ in range(8)]
            torch.cuda.synchronize()
            a.record(stream)
            facs32 = rcp.factor_batch([p] * 16, eps_16, rcp.RCP_FP32_REFINED, buffers=list(bufs) + more)
            b.record(stream)
            torch.cuda.synchronize()
            t_b32x2 = a.elapsed_time(b) * 1e-3
            del facs32, eps_16, more
            torch.cuda.empty_cache()
        fac = rcp.Factors(p, eps, rcp.RCP_FP64, buffer=buf)
        F64, z64 = rcp.reciprocal_average(fac, p, want_z=True)
        torch.cuda.synchronize()
        zerr = (torch.linalg.vector_norm(z32 - z64) / torch.linalg.vector_norm(z64)).item()
        out["fp32_refined"] = {"lu_single": {"seconds": round(t_f32, 5),
                                             **lu_rates(p, t_f32, 1, FP32_PEAK_TFLOPS)},
                               "refine_steps": it, "rel_residual": res,
                               "field_rel_err_vs_fp64": zerr,
                               "F_rel_err_vs_fp64": abs(F32.item() - F64.item()) / abs(F64.item())}
        if t_b32 is not None:
            out["fp32_refined"]["lu_batch"] = {
                "geometries": B, "seconds": round(t_b32, 5),
                **lu_rates(p, t_b32, B, FP32_PEAK_TFLOPS),
                "speedup_vs_fp64_batch": round(out["lu_batch"]["seconds"] / t_b32, 3)
                if "lu_batch" in out else None}
        if t_b32x2 is not None:
            out["fp32_refined"]["lu_batch16"] = {
                "geometries": 16, "groups": "two groups of 8, each on a stream of the library",
                "seconds": round(t_b32x2, 5), **lu_rates(p, t_b32x2, 16, FP32_PEAK_TFLOPS),
                "speedup_vs_fp64_batch_per_geometry":
                    round(out["lu_batch"]["seconds"] / 8 / (t_b32x2 / 16), 3) if "lu_batch" in out else None}
        log(f"fp32 refined: factor {t_f32 * 1e3:.1f} ms, {it} steps, field err {zerr:.2e}")
        del f32, buf32
        # broadband: the geometry at the eight wavelengths of a flat spectral rule
        if args.broadband > 0 and B >= args.broadband:
            del fac
            out["broadband"] = broadband_extra(args, rcp, W, p, widths[-1], bufs, stream)
            log(f"broadband: {out['broadband']}")
        # inverse design: B seeded designs, L-BFGS-B each, evaluations batched
        if args.design_iters > 0:
            out["design"] = design_extra(args, W, p, B, bufs)
            log(f"design: {out['design']}")
    # the step's factor buffers are not needed any more: serving gets the memory
    results = fac = bufs = buf = bufsets = None
    if not args.no_extras and args.threed:
        import torch
        torch.cuda.empty_cache()
        out["threed"] = threed_extra(args)
        log(f"3d: {out['threed']}")
    if args.serve_requests > 0:
        out["serving"] = serving(args)
        out["p50_ms"] = out["serving"]["p50_ms"]
        out["p99_ms"] = out["serving"]["p99_ms"]
        out["config"]["serving"] = out["serving"]["stream"]
        log(f"serving: {out['serving']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the workload itself, ~1 min) ...")
        out["cpu_baseline"] = cpu_baseline(replace(p, widths=W.seeded_widths(len(p.widths), 1002)))
        log(f"cpu baseline {out['cpu_baseline']['value']:.4g} evals/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

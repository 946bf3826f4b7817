"""Benchmark of the SIPG multigrid hot path on one MI355X.

A step is one GMG-preconditioned CG solve to relative residual 1e-10 of the
3-D Poisson problem -Laplace u = f on the unit cube, f = 3 pi^2 prod sin(pi x_i)
(load b = M I_h f), SIPG Q3 on 32^3 cells (2,097,152 DoFs, 5 levels), FP64
throughout: every step runs the whole path (apply, colourised patch smoother
by fast diagonalisation, residual + restriction, prolongation, coarse solve,
V-cycle, PCG) with inputs resident in HBM.  `value` is solved DoFs per second
(ndofs / time per solve).

Also reported: apply and smoothing-step throughput (GDoF/s) measured with HIP
events on the library's stream, the mixed-precision (FP32 V-cycle) solve on
the same problem, the roofline position of the dominant kernel (the patch
smoother on the finest level), the Full vertex-patch kernel's smoothing step
and solve on the same problem, time to solution of the 3-D Q7 64^3 problem
(134M DoFs) all-FP64 vs mixed and of 16 batched right-hand sides (3-D Q4 32^3)
vs 16 single FP64 solves, and the FP64 CPU oracle timed on a bounded sample of
the bench workload.  Kernel workgroup shapes are autotuned before timing.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s of SIPG apply & patch smoother; time-to-1e-10 solve, FP64 vs mixed"
CAL_BYTES = 32 * 1024 * 1024
KERNEL_SRC = os.path.join(ROOT, "paper_2405_18982_amd", "csrc", "dgmg_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_smooth_poisson3d_q3_32c_traffic.txt")


def traffic_from_profile():
    """HBM bytes per finest-level smoother launch from the committed counter
    summary, if it was taken on the current kernel source; else None."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return None
    src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    vals = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line:
            key, val = line.split(":", 1)
            vals[key.strip()] = val.strip()
    if vals.get("kernel_source_sha256") != src:
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
WORKLOAD = "poisson3d_q3_32c"


def cpu_baseline(dim, k, L, sigma, iters_gpu, budget_iters=2):
    """Time the oracle's own PCG (matrix-free Kronecker apply, FD smoother,
    V-cycle) on the host for a bounded number of iterations and scale to the
    GPU's iteration count.  The oracle builds its own load vector."""
    from oracle.multigrid import Hierarchy
    from oracle.rhs import interpolate
    from oracle.sipg import mass_operator
    from paper_2405_18982_amd import inputs
    N = 2 ** (L + 1)
    b_host = mass_operator(dim, k, N) @ interpolate(dim, k, N, inputs.sine_load)
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    H = Hierarchy(dim, k, L, sigma)
    t_setup = time.perf_counter() - t0
    A = H.apply[L]
    r = b_host.copy()
    x = np.zeros_like(r)
    t0 = time.perf_counter()
    z = H.vcycle(r)
    p = z.copy()
    rz = r @ z
    for _ in range(budget_iters):
        q = A(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = H.vcycle(r)
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    t_iter = (time.perf_counter() - t0) / (budget_iters + 1)
    t_solve = t_iter * (iters_gpu + 1)
    ndof = b_host.size
    return {
        "value": ndof / t_solve / 1e9,
        "unit": "GDoF/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"{budget_iters} oracle PCG iterations plus the initial V-cycle on the same "
                   f"workload ({t_iter:.2f} s per iteration), scaled to the GPU's {iters_gpu} "
                   f"iterations; oracle setup {t_setup:.1f} s not counted"),
        "seconds_per_solve_est": t_solve,
    }


def _time_solves(prob, b, reps, warm=1):
    import torch
    x = torch.empty_like(b)
    for _ in range(warm):
        prob.solve(b, rtol=1e-10, maxit=100, out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, it, rel = prob.solve(b, rtol=1e-10, maxit=100, out=x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps, it, rel, x


def bench_q7_mixed(reps=2):
    """3-D Q7 64^3 (134M DoFs), b ~ U[-1,1] seed 3: all-FP64 solve vs FP32
    V-cycle inside FP64 CG, same GPU, time to 1e-10."""
    import torch
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS["poisson3d_q7_64c_mixed"]
    res, xs = {}, {}
    for prec in (64, 32):
        p = dgmg.Problem(w["dim"], w["k"], w["L"], precision=prec)
        p.autotune(nrhs=1)
        b = torch.from_numpy(inputs.uniform(w["seed"], p.ndofs())).cuda()
        t, it, rel, x = _time_solves(p, b, reps)
        res[f"fp{prec}_ms"] = t * 1e3
        res[f"fp{prec}_iterations"] = int(it[0])
        xs[prec] = x.clone()
        p.close()
        del b, x
    res["mixed_speedup"] = res["fp64_ms"] / res["fp32_ms"]
    res["mixed_vs_fp64_rel_diff"] = float(torch.linalg.norm(xs[32] - xs[64]) / torch.linalg.norm(xs[64]))
    res["ndofs"] = int(xs[64].numel())
    del xs
    torch.cuda.empty_cache()
    return res


def bench_batched(reps=3):
    """3-D Q4 32^3, 16 right-hand sides N(0,1) seed 4 solved together (FP32
    V-cycle in FP64 CG, one launch per kernel for all 16, captured V-cycle,
    autotuned shapes) vs 16 separate all-FP64 solves."""
    import torch
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS["poisson3d_q4_32c_16rhs"]
    pm = dgmg.Problem(w["dim"], w["k"], w["L"], precision=32, nrhs_max=w["nrhs"])
    tuned = pm.autotune(nrhs=w["nrhs"])
    B = torch.from_numpy(inputs.normal(w["seed"], (w["nrhs"], pm.ndofs()))).cuda()
    tb, itb, _, xb = _time_solves(pm, B, reps)
    p64 = dgmg.Problem(w["dim"], w["k"], w["L"], precision=64)
    p64.autotune(nrhs=1)
    ts, its = 0.0, []
    x1 = torch.empty_like(B)
    for j in range(w["nrhs"]):
        t, it, _, x = _time_solves(p64, B[j].contiguous(), 1, warm=1 if j == 0 else 0)
        ts += t
        its.append(int(it[0]))
        x1[j] = x
    out = {"ndofs_per_rhs": pm.ndofs(), "nrhs": w["nrhs"], "batched_mixed_ms": tb * 1e3,
           "batched_iterations": [int(i) for i in itb], "single_fp64_total_ms": ts * 1e3,
           "single_iterations": its, "speedup": ts / tb,
           "rel_diff_vs_fp64": float(torch.linalg.norm(xb - x1) / torch.linalg.norm(x1)),
           "tuned": tuned.strip().splitlines()}
    pm.close()
    p64.close()
    return out


def bench_adjoint(reps=3):
    """2-D Q5 256^2 (2.4M DoFs), kappa = 1: the differentiable solve, loss
    1/2 |u - u_t|^2 with load and target interpolated from seeded Fourier
    fields; forward solve and backward (adjoint solve + dL/dkappa) timed
    separately, tolerance 1e-10."""
    import torch
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS["poisson2d_q5_256c_adjoint"]
    prob = dgmg.Problem(w["dim"], w["k"], w["L"], kappa=w["kappa"])
    prob.autotune(nrhs=1)
    X = prob.node_coords()
    b = prob.mass(torch.from_numpy(inputs.fourier_field(inputs.fourier_modes(w["seed"]), X)).cuda())
    ut = torch.from_numpy(inputs.fourier_field(inputs.fourier_modes(w["target_seed"]), X)).cuda()
    tf = tb = 0.0
    for rep in range(reps + 1):
        bb = b.clone().requires_grad_(True)
        kap = torch.tensor(w["kappa"], dtype=torch.float64, device="cuda", requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = dgmg.solve(bb, kap, prob, rtol=1e-10)
        loss = 0.5 * ((u - ut) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep > 0:  # the first pass warms up
            tf += t1 - t0
            tb += t2 - t1
    out = {"ndofs": prob.ndofs(), "forward_ms": tf / reps * 1e3, "backward_ms": tb / reps * 1e3,
           "dloss_dkappa": float(kap.grad), "grad_b_norm": float(torch.linalg.norm(bb.grad))}
    prob.close()
    return out


def bench_full_kernel(b, xin, t_smooth_dirichlet, ms_dirichlet, reps=5):
    """The Full vertex-patch kernel (whole patch, residual once per colour) on
    the bench workload: smoothing-step time against the Dirichlet kernel's
    (the paper measures the Full step 4-5x slower) and the time to 1e-10."""
    import torch
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS[WORKLOAD]
    pf = dgmg.Problem(w["dim"], w["k"], w["L"], variant=dgmg.SMOOTH_FULL)
    tuned = pf.autotune(nrhs=1)
    xs = xin.clone()
    pf.smooth(xs, b)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        pf.smooth(xs, b)
    e1.record()
    e1.synchronize()
    t_step = e0.elapsed_time(e1) * 1e-3 / 20
    t, it, rel, _ = _time_solves(pf, b, reps)
    pf.close()
    return {"smooth_step_us": t_step * 1e6, "step_vs_dirichlet": t_step / t_smooth_dirichlet,
            "ms_per_solve": t * 1e3, "pcg_iterations": int(it[0]),
            "solve_vs_dirichlet": t * 1e3 / ms_dirichlet, "tuned": tuned.strip().splitlines()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3-D Q7 mixed, the batched 16-RHS and the 2-D adjoint runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (--gpus 1); it has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2405_18982_amd import dgmg, inputs, roofline

    w = inputs.WORKLOADS[WORKLOAD]
    dim, k, L = w["dim"], w["k"], w["L"]
    sigma = inputs.sigma_of(k)
    N = 2 ** (L + 1)
    prob = dgmg.Problem(dim, k, L, sigma=sigma)
    tuned = prob.autotune(nrhs=1)
    ndof = prob.ndofs()
    b = prob.mass(torch.from_numpy(inputs.sine_load(prob.node_coords())).cuda())
    x = torch.empty_like(b)
    rtol = 1e-10

    def solve():
        return prob.solve(b, rtol=rtol, maxit=100, out=x)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, it, rel = solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    iters = int(it[0])
    value = ndof / (ms * 1e-3) / 1e9

    # component throughput with HIP events on the library's (torch's current) stream
    def timed(fn, reps):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    # calibration copy of a known size: the HBM counters of this plain copy
    # kernel scale the smoother's counters to bytes (see traffic_from_profile)
    cal_src = torch.ones(CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    xin = torch.from_numpy(inputs.uniform(w["seed"], ndof)).cuda()
    yout = torch.empty_like(xin)
    t_apply = timed(lambda: prob.apply(xin, out=yout), 50)
    xs = xin.clone()
    t_smooth = timed(lambda: prob.smooth(xs, b), 20)
    nc = 2 ** dim
    sc = roofline.smooth_step_counts(dim, k, N)
    ac = roofline.apply_counts(dim, k, N)
    rf = roofline.bound(sc, t_smooth, precision=64)
    roof = {
        "kernel": "k_smooth (FP64, exact residual) on the finest level, 8 colour launches per step",
        "bound": rf["bound"], "achieved": round(rf["achieved"], 2), "peak": rf["peak"],
        "unit": rf["unit"], "frac": round(rf["frac"], 4), "traffic": traffic_from_profile(),
        "algorithmic_bytes_per_launch": sc["bytes"] / nc,
        "algorithmic_flops_per_launch": sc["flops"] / nc,
        "avg_launch_us": t_smooth / nc * 1e6,
        "achieved_tflops": round(rf.get("achieved_tflops", rf["achieved"]), 3),
    }
    ra = roofline.bound(ac, t_apply, precision=64)
    components = {
        "apply_gdofs": ndof / t_apply / 1e9,
        "apply_us": t_apply * 1e6,
        "apply_roofline": {"bound": ra["bound"], "achieved": round(ra["achieved"], 2),
                           "unit": ra["unit"], "frac": round(ra["frac"], 4)},
        "smooth_gdofs": ndof / t_smooth / 1e9,
        "smooth_step_us": t_smooth * 1e6,
        "tuned": tuned.strip().splitlines(),
        "pcg_iterations": iters,
        "final_relres": float(rel[0]),
        "fp64_ms_per_solve": ms,
    }

    if not args.no_mixed:
        pm = dgmg.Problem(dim, k, L, sigma=sigma, precision=dgmg.FP32)
        pm.autotune(nrhs=1)
        xm = torch.empty_like(b)
        for _ in range(args.warmup):
            pm.solve(b, rtol=rtol, maxit=100, out=xm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, itm, relm = pm.solve(b, rtol=rtol, maxit=100, out=xm)
        torch.cuda.synchronize()
        msm = (time.perf_counter() - t0) * 1e3 / args.steps
        xs32, b32 = xs.float(), b.float()
        t_smooth32 = timed(lambda: pm.smooth(xs32, b32), 20)
        components.update({
            "mixed_ms_per_solve": msm,
            "mixed_iterations": int(itm[0]),
            "mixed_speedup_vs_fp64": ms / msm,
            "mixed_vs_fp64_rel_diff": float(torch.linalg.norm(xm - x) / torch.linalg.norm(x)),
            "smooth_fp32_gdofs": ndof / t_smooth32 / 1e9,
        })
        pm.close()

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDoF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "dim": dim, "degree": k, "cells_per_dir": N,
                   "levels": L + 1, "ndofs": ndof, "penalty_sigma": sigma, "rtol": rtol,
                   "step": "one GMG-PCG solve to relative residual 1e-10",
                   "parallelism": "single GPU"},
        "roofline": roof,
        "components": components,
    }
    if not args.no_extra:
        components["full_kernel"] = bench_full_kernel(b, xin, t_smooth, ms)
        components["q7_64c_fp64_vs_mixed"] = bench_q7_mixed()
        components["q4_32c_16rhs_batched"] = bench_batched()
        components["q5_256c_2d_adjoint"] = bench_adjoint()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(dim, k, L, sigma, iters)
    prob.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

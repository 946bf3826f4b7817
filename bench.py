"""Benchmark of the SIPG multigrid hot path on one MI355X.

A step is one GMG-preconditioned CG solve to relative residual 1e-10 of the
3-D Poisson problem -Laplace u = f on the unit cube, f = 3 pi^2 prod sin(pi x_i)
(load b = M I_h f), SIPG Q3 on 32^3 cells (2,097,152 DoFs, 5 levels), FP64
throughout: every step runs the whole path (apply, colourised patch smoother
by fast diagonalisation, residual + restriction, prolongation, coarse solve,
V-cycle, PCG) with inputs resident in HBM.  `value` is solved DoFs per second
(ndofs / time per solve).

Also reported, per workload (`components`): the finest-level apply and one
smoothing step (all colours) in FP64 and FP32, each with HIP-event timings on
the library's stream and its roofline position (algorithmic bytes and flops
of `roofline.py` against the MI355X peaks); FP64 against mixed-precision (FP32
V-cycle) time to solution on the 2.1M-DoF and the 134M-DoF (3-D Q7 64^3)
problems; 16 batched right-hand sides (3-D Q4 32^3) against 16 single solves
in the same precision (FP64 and mixed); the differentiable 2-D Q5 256^2
solve; the Full vertex-patch kernel.  The oracle leg times the FP64 CPU
oracle on the host (`cpu_baseline`) and, having the oracle's exact discrete
solutions at hand, states the error of the GPU's FP64 and mixed solutions
against them (`error_vs_oracle_exact`).  Kernel shapes are autotuned first.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
    python bench.py --cpu-full     # the oracle alone, every workload, all
                                   # cores and 1 thread (minutes; no GPU)
"""
import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GDoF/s of SIPG apply & patch smoother; time-to-1e-10 solve, FP64 vs mixed"
CAL_BYTES = 32 * 1024 * 1024
KERNEL_SRC = os.path.join(ROOT, "paper_2405_18982_amd", "csrc", "dgmg_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_smooth_poisson3d_q3_32c_traffic.txt")
WORKLOAD = "poisson3d_q3_32c"


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


# ------------------------------------------------------------------ GPU legs
def _events_time(fn, reps):
    """Mean seconds per call of fn over reps calls, HIP events on torch's
    current stream (the stream the library enqueues on)."""
    import torch
    fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / reps


def _roof(counts, seconds, precision, ndof_total):
    from paper_2405_18982_amd import roofline
    r = roofline.bound(counts, seconds, precision=precision)
    out = {"us": round(seconds * 1e6, 3), "gdofs": round(ndof_total / seconds / 1e9, 3),
           "bound": r["bound"], "achieved": round(r["achieved"], 2), "unit": r["unit"],
           "frac": round(r["frac"], 4), "ai_flop_per_byte": round(r["ai"], 2)}
    if r["bound"] == "hbm":
        out["achieved_tflops"] = round(r["achieved_tflops"], 3)
    else:
        out["achieved_gbs"] = round(r["achieved_gbs"], 1)
    return out


def kernel_rooflines(prob, nrhs, precisions=(64, 32), seed=7, reps_apply=20, reps_smooth=5):
    """Finest-level apply and one smoothing step (all colours) of `prob` in
    each precision on nrhs right-hand sides x, b ~ U[-1,1]: HIP-event time
    and roofline position of each."""
    import torch
    from paper_2405_18982_amd import inputs, roofline
    dim, k, L = prob.dim, prob.k, prob.L
    N = 2 ** (L + 1)
    n = prob.ndofs()
    shape = (nrhs, n) if nrhs > 1 else (n,)
    out = {}
    for prec in precisions:
        dt = torch.float64 if prec == 64 else torch.float32
        s = 8 if prec == 64 else 4
        x = torch.from_numpy(inputs.uniform(seed, shape)).to(device="cuda", dtype=dt)
        b = torch.from_numpy(inputs.uniform(seed + 1, shape)).to(device="cuda", dtype=dt)
        y = torch.empty_like(x)
        ta = _events_time(lambda: prob.apply(x, out=y), reps_apply)
        ts = _events_time(lambda: prob.smooth(x, b), reps_smooth)
        out[f"apply_fp{prec}"] = _roof(roofline.apply_counts(dim, k, N, nrhs, s), ta, prec, nrhs * n)
        out[f"smooth_step_fp{prec}"] = _roof(roofline.smooth_step_counts(dim, k, N, nrhs, s), ts, prec,
                                             nrhs * n)
        del x, b, y
    torch.cuda.empty_cache()
    return out


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
    V-cycle inside FP64 CG, same GPU, time to 1e-10; apply and smoothing step
    rooflines in both precisions.  Returns (results, {precision: solution on
    the host})."""
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
        res[f"fp{prec}_relres"] = float(rel[0])
        xs[prec] = x.cpu().numpy()
        del b, x
        torch.cuda.empty_cache()
        # kernels of the V-cycle's precision on its tuned shapes
        res.update(kernel_rooflines(p, 1, precisions=(prec,), reps_apply=5, reps_smooth=2))
        p.close()
    res["mixed_speedup"] = res["fp64_ms"] / res["fp32_ms"]
    res["mixed_vs_fp64_rel_diff"] = float(np.linalg.norm(xs[32] - xs[64]) / np.linalg.norm(xs[64]))
    res["ndofs"] = int(xs[64].size)
    return res, xs


def bench_batched(reps=3):
    """3-D Q4 32^3, 16 right-hand sides N(0,1) seed 4 solved together (one
    launch per kernel for all 16, captured V-cycle, autotuned shapes) against
    16 separate solves, in the same precision: FP64 V-cycle and FP32 V-cycle
    (mixed), each inside FP64 CG; batched apply and smoothing-step rooflines.
    Returns (results, {precision: batched solution on the host})."""
    import torch
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS["poisson3d_q4_32c_16rhs"]
    nr = w["nrhs"]
    out, sols = {"nrhs": nr}, {}
    B = None
    for prec, tag in ((64, "fp64"), (32, "mixed")):
        pb = dgmg.Problem(w["dim"], w["k"], w["L"], precision=prec, nrhs_max=nr)
        tuned = pb.autotune(nrhs=nr)
        if B is None:
            B = torch.from_numpy(inputs.normal(w["seed"], (nr, pb.ndofs()))).cuda()
            out["ndofs_per_rhs"] = pb.ndofs()
        tb, itb, _, xb = _time_solves(pb, B, reps)
        if prec == 32:
            out["kernels_16rhs"] = kernel_rooflines(pb, nr, reps_apply=5, reps_smooth=2)
            out["tuned_16rhs_mixed"] = tuned.strip().splitlines()
        pb.close()
        ps = dgmg.Problem(w["dim"], w["k"], w["L"], precision=prec)
        ps.autotune(nrhs=1)
        ts, its = 0.0, []
        x1 = torch.empty_like(B)
        for j in range(nr):
            t, it, _, x = _time_solves(ps, B[j].contiguous(), 1, warm=1 if j == 0 else 0)
            ts += t
            its.append(int(it[0]))
            x1[j] = x
        ps.close()
        out[f"batched_{tag}_ms"] = tb * 1e3
        out[f"batched_{tag}_iterations"] = sorted(set(int(i) for i in itb))
        out[f"single_{tag}_total_ms"] = ts * 1e3
        out[f"single_{tag}_iterations"] = sorted(set(its))
        out[f"batching_speedup_{tag}"] = ts / tb
        out[f"batched_vs_single_rel_diff_{tag}"] = float(torch.linalg.norm(xb - x1) / torch.linalg.norm(x1))
        sols[prec] = xb.cpu().numpy()
        del xb, x1
        torch.cuda.empty_cache()
    out["batched_mixed_vs_16_single_fp64"] = out["single_fp64_total_ms"] / out["batched_mixed_ms"]
    return out, sols


def bench_adjoint(reps=3):
    """2-D Q5 256^2 (2.4M DoFs), kappa = 1: the differentiable solve, loss
    1/2 |u - u_t|^2 with load and target interpolated from seeded Fourier
    fields; forward solve and backward (adjoint solve + dL/dkappa) timed
    separately, tolerance 1e-10; apply and smoothing-step rooflines.
    Returns (results, host copies of b and u)."""
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
    out.update(kernel_rooflines(prob, 1, precisions=(64,)))
    host = {"b": b.cpu().numpy(), "u": u.detach().cpu().numpy()}
    prob.close()
    return out, host


def bench_full_kernel(b, xin, t_smooth_dirichlet, ms_dirichlet, reps=5):
    """The Full vertex-patch kernel (whole patch, residual once per colour) on
    the bench workload: smoothing-step time against the Dirichlet kernel's
    (the paper measures the Full step 4-5x slower) and the time to 1e-10."""
    from paper_2405_18982_amd import dgmg, inputs
    w = inputs.WORKLOADS[WORKLOAD]
    pf = dgmg.Problem(w["dim"], w["k"], w["L"], variant=dgmg.SMOOTH_FULL)
    tuned = pf.autotune(nrhs=1)
    xs = xin.clone()
    t_step = _events_time(lambda: pf.smooth(xs, b), 20)
    t, it, rel, _ = _time_solves(pf, b, reps)
    pf.close()
    return {"smooth_step_us": t_step * 1e6, "step_vs_dirichlet": t_step / t_smooth_dirichlet,
            "ms_per_solve": t * 1e3, "pcg_iterations": int(it[0]),
            "solve_vs_dirichlet": t * 1e3 / ms_dirichlet, "tuned": tuned.strip().splitlines()}


# ---------------------------------------------------------------- oracle leg
def _host_info():
    model = platform.processor() or ""
    try:
        p = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10)
        for line in p.stdout.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except Exception:
        avail = os.cpu_count() or 1
    return model, os.cpu_count() or 1, avail


def _pool_threads():
    try:
        from threadpoolctl import threadpool_info
        return max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def _median_time(fn, reps=5, warm=1):
    for _ in range(warm):
        fn()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def _oracle_problem(name):
    """Oracle hierarchy and load vector of a workload, built by the oracle
    from the same seeded inputs as the GPU side."""
    from oracle.multigrid import Hierarchy
    from oracle.rhs import interpolate, node_coords
    from oracle.sipg import mass_operator
    from paper_2405_18982_amd import inputs
    w = inputs.WORKLOADS[name]
    d, k, L = w["dim"], w["k"], w["L"]
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    H = Hierarchy(d, k, L, sig, kappa=w["kappa"])
    if w["rhs"] == "sine":
        b = mass_operator(d, k, N) @ interpolate(d, k, N, inputs.sine_load)
    elif w["rhs"] == "fourier":
        X = node_coords(d, k, N)
        b = mass_operator(d, k, N) @ inputs.fourier_field(inputs.fourier_modes(w["seed"]), X)
    elif w["rhs"] == "uniform":
        b = inputs.uniform(w["seed"], H.ndofs(L))
    else:
        b = inputs.normal(w["seed"], (w["nrhs"], H.ndofs(L)))
    return H, b, w


def _oracle_solve_seconds(H, b, reps, warm):
    from oracle.multigrid import pcg
    L = H.L
    res = {}

    def run():
        x, it, _, rel = pcg(H.apply[L], H.vcycle, b, rtol=1e-10, maxit=100)
        res.update(it=it, rel=rel)

    t = _median_time(run, reps, warm)
    return t, res["it"], res["rel"]


def cpu_baseline(gpu_solutions):
    """The oracle leg (host only).  Times the FP64 oracle's own PCG
    (oracle.multigrid.pcg: matrix-free Kronecker apply, FD smoother, V-cycle)
    to 1e-10 on the bench workload, median of 3 solves after one warm-up, on
    the host's cores through NumPy's thread pools; the oracle's apply,
    smoothing step and V-cycle alone as medians of 5 after one warm-up.
    Then the oracle's exact discrete solutions (global fast diagonalisation)
    of the workloads whose GPU solutions are passed in, and the relative error
    of each GPU solution against them."""
    from oracle.fdsolve import GlobalFD
    from paper_2405_18982_amd import inputs
    model, ncpu, avail = _host_info()
    H, b, w = _oracle_problem(WORKLOAD)
    L = H.L
    ndof = b.size
    x = inputs.uniform(7, ndof)
    t_apply = _median_time(lambda: H.apply[L](x))
    t_smooth = _median_time(lambda: H.smooth(L, x, b, H.asc))
    t_vc = _median_time(lambda: H.vcycle(b))
    t_solve, it, rel = _oracle_solve_seconds(H, b, reps=3, warm=1)
    base = {
        "value": ndof / t_solve / 1e9, "unit": "GDoF/s", "cores": _pool_threads(), "kind": "oracle",
        "sample": (f"oracle.multigrid.pcg to 1e-10 on the bench workload (3-D Q3 32^3, 2.1M DoFs): "
                   f"median of 3 solves after 1 warm-up, {it} iterations, {t_solve:.2f} s per solve; "
                   f"NumPy/BLAS thread pools at their default size; oracle setup not counted"),
        "cpu_model": model, "host_cpus": ncpu, "affinity_cpus": avail,
        "seconds_per_solve": t_solve, "oracle_iterations": int(it), "oracle_true_relres": float(rel),
        "apply_ms": t_apply * 1e3, "smooth_step_ms": t_smooth * 1e3, "vcycle_ms": t_vc * 1e3,
        "apply_gdofs": ndof / t_apply / 1e9, "smooth_step_gdofs": ndof / t_smooth / 1e9,
        "timing": "time.perf_counter, median of 5 after 1 warm-up (apply, smoothing step, V-cycle)",
    }
    errs = {}
    for name, sols in gpu_solutions.items():
        wk = inputs.WORKLOADS[name]
        d, k, Lw = wk["dim"], wk["k"], wk["L"]
        fd = GlobalFD(d, k, 2 ** (Lw + 1), inputs.sigma_of(k), wk["kappa"])
        bw = sols.pop("b")
        ex = fd.solve(bw) if bw.ndim == 1 else np.stack([fd.solve(r) for r in bw])
        e = {}
        for tag, u in sols.items():
            e[tag] = float(np.linalg.norm(u - ex) / np.linalg.norm(ex))
        errs[name] = e
        del ex
    return base, errs


def cpu_full():
    """Every workload on the oracle alone, with all host cores and with one
    thread (NumPy/BLAS pools limited by threadpoolctl): full PCG solves of
    the 2-D Q2 8x8, 3-D Q3 32^3 and 2-D Q5 256^2 problems (median of 5 after
    1 warm-up); apply and smoothing step of the 3-D Q4 32^3 problem for one
    and for 16 right-hand sides; apply and one smoothing step of the 3-D Q7
    64^3 problem, the smoothing step over a chunk of the colours' patches
    (one colour) scaled by the colour count."""
    from threadpoolctl import threadpool_limits
    from paper_2405_18982_amd import inputs
    model, ncpu, avail = _host_info()
    out = {"cpu_model": model, "host_cpus": ncpu, "affinity_cpus": avail, "rows": []}

    def emit(row):
        out["rows"].append(row)
        print(json.dumps(row), flush=True)

    for name in ("poisson2d_q2_8x8", WORKLOAD, "poisson2d_q5_256c_adjoint"):
        H, b, w = _oracle_problem(name)
        for thr in (None, 1):
            print(f"# {name} oracle PCG solves, threads={thr}", flush=True)
            with threadpool_limits(limits=thr):
                t, it, rel = _oracle_solve_seconds(H, b, reps=5, warm=1)
                emit({"workload": name, "what": "pcg solve to 1e-10", "threads": thr or _pool_threads(),
                      "seconds": t, "iterations": int(it), "gdofs": b.size / t / 1e9})
        del H, b
    H, B, w = _oracle_problem("poisson3d_q4_32c_16rhs")
    L = H.L
    X = inputs.uniform(7, B.shape)
    for thr in (None, 1):
        with threadpool_limits(limits=thr):
            for nr in (1, 16):
                print(f"# 3-D Q4 32^3 oracle apply and smoothing step, nrhs={nr}, threads={thr}", flush=True)
                ta = _median_time(lambda: [H.apply[L](X[j]) for j in range(nr)], reps=5 if nr == 1 else 3)
                ts = _median_time(lambda: [H.smooth(L, X[j], B[j], H.asc) for j in range(nr)],
                                  reps=5 if nr == 1 else 3)
                emit({"workload": "poisson3d_q4_32c_16rhs", "nrhs": nr, "threads": thr or _pool_threads(),
                      "apply_s": ta, "smooth_step_s": ts, "apply_gdofs": nr * B.shape[1] / ta / 1e9,
                      "smooth_step_gdofs": nr * B.shape[1] / ts / 1e9})
    del H, B, X
    from oracle.sipg import KronApply
    from oracle.smoother import FDSmoother
    w = inputs.WORKLOADS["poisson3d_q7_64c_mixed"]
    d, k, L = w["dim"], w["k"], w["L"]
    N = 2 ** (L + 1)
    sig = inputs.sigma_of(k)
    ap = KronApply(d, k, N, sig)
    sm = FDSmoother(d, k, N, sig, 1.0, "exact", ap)
    n = (N * (k + 1)) ** d
    x = inputs.uniform(7, n)
    b = inputs.uniform(3, n)
    for thr in (None, 1):
        with threadpool_limits(limits=thr):
            print(f"# 3-D Q7 64^3 oracle apply and colour-0 sweep, threads={thr}", flush=True)
            ta = _median_time(lambda: ap(x), reps=3)
            tc = _median_time(lambda: sm.step(x, b, [0]), reps=1, warm=0)
            emit({"workload": "poisson3d_q7_64c_mixed", "threads": thr or _pool_threads(), "apply_s": ta,
                  "smooth_colour0_s": tc, "smooth_step_est_s": tc * 2 ** d,
                  "note": "smoothing step estimated as 8 x the colour-0 sweep (colours have "
                          "equal patch counts up to the boundary layer)",
                  "apply_gdofs": n / ta / 1e9})
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the 3-D Q7 mixed, the batched 16-RHS, the 2-D adjoint and Full runs")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle alone on every workload (host only) and exit")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (--gpus 1); it has no multi-GPU "
              "path", file=sys.stderr)
        sys.exit(2)
    if args.cpu_full:
        cpu_full()
        return

    import torch

    from paper_2405_18982_amd import dgmg, inputs, roofline

    w = inputs.WORKLOADS[WORKLOAD]
    dim, k, L = w["dim"], w["k"], w["L"]
    sigma = inputs.sigma_of(k)
    N = 2 ** (L + 1)
    torch.zeros(1, device="cuda")  # the GPU context and the library load are not
    dgmg.lib()                     # part of the set-up time
    torch.cuda.synchronize()
    t_setup = time.perf_counter()
    prob = dgmg.Problem(dim, k, L, sigma=sigma)
    torch.cuda.synchronize()
    t_tune = time.perf_counter()
    tuned = prob.autotune(nrhs=1)
    torch.cuda.synchronize()
    t_tuned = time.perf_counter()
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

    # calibration copy of a known size: the HBM counters of this plain copy
    # kernel scale the smoother's counters to bytes (see traffic_from_profile)
    cal_src = torch.ones(CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    torch.cuda.synchronize()
    xin = torch.from_numpy(inputs.uniform(w["seed"], ndof)).cuda()
    yout = torch.empty_like(xin)
    t_apply = _events_time(lambda: prob.apply(xin, out=yout), 50)
    xs = xin.clone()
    t_smooth = _events_time(lambda: prob.smooth(xs, b), 20)
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
    c2 = {
        "apply_fp64": _roof(ac, t_apply, 64, ndof),
        "smooth_step_fp64": _roof(sc, t_smooth, 64, ndof),
        "tuned": tuned.strip().splitlines(),
        "pcg_iterations": iters,
        "final_relres": float(rel[0]),
        "fp64_ms_per_solve": ms,
        # not part of the solve: mesh, tables, level vectors and the dense
        # bottom operator (set-up), and the shape search (autotune)
        "setup_ms": round((t_tune - t_setup) * 1e3, 2),
        "autotune_ms": round((t_tuned - t_tune) * 1e3, 2),
    }
    # one V-cycle with the bottom levels as the dense operator (the solve's
    # setting) and as the fused bottom launch
    xv = torch.empty_like(b)
    t_vc = _events_time(lambda: prob.vcycle(b, out=xv), 30)
    prob.use_dense_bottom(False)
    t_vc_launch = _events_time(lambda: prob.vcycle(b, out=xv), 30)
    prob.use_dense_bottom(True)
    c2["vcycle_us"] = {"dense_bottom": round(t_vc * 1e6, 2), "bottom_launch": round(t_vc_launch * 1e6, 2),
                       "dense_bottom_level": prob.dense_bottom_level()}
    c2.update({k2: v for k2, v in kernel_rooflines(prob, 1, precisions=(32,)).items()})
    components = {WORKLOAD: c2}
    host_sols = {WORKLOAD: {"b": b.cpu().numpy(), "gpu_fp64": x.cpu().numpy()}}

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
        c2.update({
            "mixed_ms_per_solve": msm,
            "mixed_iterations": int(itm[0]),
            "mixed_relres": float(relm[0]),
            "mixed_speedup_vs_fp64": ms / msm,
            "mixed_vs_fp64_rel_diff": float(torch.linalg.norm(xm - x) / torch.linalg.norm(x)),
        })
        host_sols[WORKLOAD]["gpu_mixed"] = xm.cpu().numpy()
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
        c2["full_kernel"] = bench_full_kernel(b, xin, t_smooth, ms)
        q7, q7x = bench_q7_mixed()
        components["poisson3d_q7_64c_mixed"] = q7
        q4, q4x = bench_batched()
        components["poisson3d_q4_32c_16rhs"] = q4
        adj, adjx = bench_adjoint()
        components["poisson2d_q5_256c_adjoint"] = adj
        wq7 = inputs.WORKLOADS["poisson3d_q7_64c_mixed"]
        host_sols["poisson3d_q7_64c_mixed"] = {"b": inputs.uniform(wq7["seed"], q7["ndofs"]),
                                               "gpu_fp64": q7x[64], "gpu_mixed": q7x[32]}
        wq4 = inputs.WORKLOADS["poisson3d_q4_32c_16rhs"]
        host_sols["poisson3d_q4_32c_16rhs"] = {
            "b": inputs.normal(wq4["seed"], (wq4["nrhs"], q4["ndofs_per_rhs"])),
            "gpu_fp64": q4x[64], "gpu_mixed": q4x[32]}
        host_sols["poisson2d_q5_256c_adjoint"] = {"b": adjx["b"], "gpu_fp64": adjx["u"]}
    prob.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["error_vs_oracle_exact"] = cpu_baseline(host_sols)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()

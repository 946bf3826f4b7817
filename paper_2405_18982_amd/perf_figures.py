"""The paper's performance measurements on one MI355X (Sec. 5): throughput of
the operator and of one smoothing step against problem size (the saturation
study of Fig. throughput_4), arithmetic throughput per component (Fig.
Arithmetic), FP32 over FP64 speedup per component and degree (Fig.
speedup_mixed), and one smoothing step and the GMRES solve per local kernel
at 134M DoFs (Fig. Smoothing).  3-D throughout, synthetic data (x, b ~
U[-1,1] seeded; f = 1 for the solves, b = M 1), times from HIP events on the
library's stream after warm-up, best of several batches.

    python -m paper_2405_18982_amd.perf_figures [throughput|arith|mixed|kernels|all]
        [--json out.jsonl]

Every arithmetic step runs in libdgmg on the GPU; this module only times it.
"""
import argparse
import json
import sys

from . import inputs, roofline


def _torch():
    import torch
    return torch


def _time(fn, reps=10, batches=3):
    torch = _torch()
    fn()
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(batches):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3 / reps)
    return best


def _vectors(prob, level, dtype, seed=11):
    torch = _torch()
    n = prob.ndofs(level)
    x = torch.from_numpy(inputs.uniform(seed, n)).to("cuda", dtype)
    b = torch.from_numpy(inputs.uniform(seed + 1, n)).to("cuda", dtype)
    return x, b


def throughput(out, k=4, levels=(2, 3, 4, 5, 6)):
    """GDoF/s of A x and of one smoothing step (FP64, FP32) against size."""
    from . import dgmg
    torch = _torch()
    for L in levels:
        N = 2 ** (L + 1)
        for prec in (64, 32):
            dt = torch.float64 if prec == 64 else torch.float32
            prob = dgmg.Problem(3, k, L, precision=prec)
            prob.autotune(nrhs=1)
            x, b = _vectors(prob, L, dt)
            y = torch.empty_like(x)
            ta = _time(lambda: prob.apply(x, out=y), reps=20)
            ts = _time(lambda: prob.smooth(x, b), reps=5)
            nd = prob.ndofs()
            r = {"fig": "throughput", "k": k, "L": L, "cells_per_dir": N, "ndofs": nd, "precision": prec,
                 "apply_us": ta * 1e6, "apply_gdofs": nd / ta / 1e9,
                 "smooth_us": ts * 1e6, "smooth_gdofs": nd / ts / 1e9}
            out(r)
            prob.close()
            del x, b, y
            torch.cuda.empty_cache()


def arith(out, k_list=(1, 2, 3, 4, 5, 6, 7), target=2 ** 27):
    """TFLOP/s and GB/s of A x and one smoothing step, FP64, about 134M DoFs."""
    from . import dgmg
    torch = _torch()
    for k in k_list:
        L = _level_for(k, target)
        N = 2 ** (L + 1)
        prob = dgmg.Problem(3, k, L)
        prob.autotune(nrhs=1)
        x, b = _vectors(prob, L, torch.float64)
        y = torch.empty_like(x)
        ta = _time(lambda: prob.apply(x, out=y), reps=10)
        ts = _time(lambda: prob.smooth(x, b), reps=3)
        ra = roofline.bound(roofline.apply_counts(3, k, N), ta)
        rs = roofline.bound(roofline.smooth_step_counts(3, k, N), ts)
        out({"fig": "arith", "k": k, "L": L, "ndofs": prob.ndofs(),
             "apply_tflops": roofline.apply_counts(3, k, N)["flops"] / ta / 1e12,
             "apply_gbs": roofline.apply_counts(3, k, N)["bytes"] / ta / 1e9, "apply_bound": ra["bound"],
             "smooth_tflops": roofline.smooth_step_counts(3, k, N)["flops"] / ts / 1e12,
             "smooth_gbs": roofline.smooth_step_counts(3, k, N)["bytes"] / ts / 1e9,
             "smooth_bound": rs["bound"]})
        prob.close()
        del x, b, y
        torch.cuda.empty_cache()


def _level_for(k, target):
    """Finest level whose DoF count is closest to target from below (>= L=2)."""
    L = 2
    while (2 ** (L + 2) * (k + 1)) ** 3 <= target:
        L += 1
    return L


def mixed(out, k_list=(1, 2, 3, 4, 5, 6, 7), target=2 ** 25):
    """FP32/FP64 time ratios of A x, one smoothing step and the GMRES solve
    (FP64 outer, V-cycle in FP32 vs FP64), about 33M DoFs per degree."""
    from . import dgmg
    torch = _torch()
    for k in k_list:
        L = _level_for(k, target)
        res = {}
        for prec in (64, 32):
            dt = torch.float64 if prec == 64 else torch.float32
            prob = dgmg.Problem(3, k, L, sigma=2.0 * k * (k + 1), precision=prec)
            prob.autotune(nrhs=1)
            x, b = _vectors(prob, L, dt)
            y = torch.empty_like(x)
            res[f"apply{prec}"] = _time(lambda: prob.apply(x, out=y), reps=10)
            res[f"smooth{prec}"] = _time(lambda: prob.smooth(x, b), reps=3)
            ones = torch.ones(prob.ndofs(), dtype=torch.float64, device="cuda")
            f1 = prob.mass(ones)
            holder = {}

            def solve():
                holder["r"] = prob.gmres(f1, rtol=1e-8, maxit=100)

            res[f"gmres{prec}"] = _time(solve, reps=1, batches=3)
            res[f"steps{prec}"] = holder["r"][1]
            prob.close()
            del x, b, y, ones, f1
            torch.cuda.empty_cache()
        out({"fig": "mixed", "k": k, "L": L, "ndofs": (2 ** (L + 1) * (k + 1)) ** 3,
             "apply_speedup": res["apply64"] / res["apply32"],
             "smooth_speedup": res["smooth64"] / res["smooth32"],
             "gmres_speedup": res["gmres64"] / res["gmres32"],
             "gmres_ms_fp64": res["gmres64"] * 1e3, "gmres_ms_mixed": res["gmres32"] * 1e3,
             "gmres_steps_fp64": res["steps64"], "gmres_steps_mixed": res["steps32"]})


def kernels(out, cases=((3, 6), (7, 5))):
    """One smoothing step and GMRES (1e-8, f = 1) per local kernel at 134M DoFs
    (3-D Q3 on 128^3 cells and Q7 on 64^3 cells), FP64."""
    from . import dgmg
    torch = _torch()
    names = {"full": dgmg.SMOOTH_FULL, "dirichlet_exact": dgmg.SMOOTH_EXACT,
             "dirichlet_paper": dgmg.SMOOTH_LOCAL, "clamped": dgmg.SMOOTH_CLAMPED}
    for k, L in cases:
        for name, var in names.items():
            prob = dgmg.Problem(3, k, L, sigma=2.0 * k * (k + 1), variant=var)
            prob.autotune(nrhs=1)
            x, b = _vectors(prob, L, torch.float64)
            ts = _time(lambda: prob.smooth(x, b), reps=2, batches=2)
            del x, b
            ones = torch.ones(prob.ndofs(), dtype=torch.float64, device="cuda")
            f1 = prob.mass(ones)
            del ones
            holder = {}

            def solve():
                holder["r"] = prob.gmres(f1, rtol=1e-8, maxit=100, raise_on_nonconvergence=False)

            tg = _time(solve, reps=1, batches=2)
            hist = holder["r"][2]
            out({"fig": "kernels", "k": k, "L": L, "ndofs": prob.ndofs(), "kernel": name,
                 "smooth_step_ms": ts * 1e3, "gmres_ms": tg * 1e3, "gmres_steps": int(holder["r"][1]),
                 "final_relres": float(hist[-1])})
            prob.close()
            del f1
            torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="?", default="all",
                    choices=["throughput", "arith", "mixed", "kernels", "all"])
    ap.add_argument("--json", default=None)
    a = ap.parse_args()
    fh = open(a.json, "w") if a.json else None

    def out(r):
        line = json.dumps(r)
        print(line, flush=True)
        if fh:
            fh.write(line + "\n")
            fh.flush()

    for name, fn in (("throughput", throughput), ("arith", arith), ("mixed", mixed), ("kernels", kernels)):
        if a.which in (name, "all"):
            print(f"# {name}", file=sys.stderr, flush=True)
            fn(out)
    if fh:
        fh.close()


if __name__ == "__main__":
    main()

"""Kernel runs for the profiler, and summaries of its counter output.

`run` drives the finest-level kernels of one workload (autotuned shapes): a
32 MiB torch copy (the calibration kernel that scales the HBM counters to
bytes), then `reps` applications of the operator and `reps` smoothing steps
in the chosen precision (with `--vcycle`: `reps` V-cycles), on x, b ~ U[-1,1]
with the workload's right-hand side count (or `--nrhs`).  Run it under
rocprofv3, e.g.

    rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_LDS -d OUT -o run --output-format csv -- \\
        python -m paper_2405_18982_amd.profile_run run --workload poisson3d_q3_32c --prec 64

`summarize` reads rocprofv3's counter CSV (one row per dispatch and counter)
and prints, per kernel name and grid size, the dispatch count and the mean
of every counter per dispatch; `summarize-trace` does the same for the
durations of a kernel-trace CSV:

    python -m paper_2405_18982_amd.profile_run summarize OUT/.../run_counter_collection.csv
    python -m paper_2405_18982_amd.profile_run summarize-trace OUT/.../run_kernel_trace.csv

Every arithmetic step runs in libdgmg on the GPU; this module only launches
it and reads the profiler's files.
"""
import argparse
import csv
import sys
from collections import defaultdict

from . import inputs

CAL_BYTES = 32 * 1024 * 1024


def run(workload, prec, reps, smooth_only=False, nrhs=None, vcycle=False):
    import torch
    from . import dgmg
    w = inputs.WORKLOADS[workload]
    nr = w["nrhs"] if nrhs is None else nrhs
    prob = dgmg.Problem(w["dim"], w["k"], w["L"], precision=prec, nrhs_max=nr)
    print(prob.autotune(nrhs=nr), flush=True)
    src = torch.ones(CAL_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    dt = torch.float64 if prec == 64 else torch.float32
    n = prob.ndofs()
    shape = (nr, n) if nr > 1 else (n,)
    x = torch.from_numpy(inputs.uniform(7, shape)).to(device="cuda", dtype=dt)
    b = torch.from_numpy(inputs.uniform(8, shape)).to(device="cuda", dtype=dt)
    y = torch.empty_like(x)
    for _ in range(reps):
        if vcycle:
            prob.vcycle(b, out=y)
            continue
        if not smooth_only:
            prob.apply(x, out=y)
        prob.smooth(x, b)
    torch.cuda.synchronize()
    what = "V-cycles" if vcycle else "reps"
    print(f"profile_run: {workload} fp{prec} nrhs={nr} {what}={reps} done", flush=True)
    prob.close()


def summarize(path, match=None):
    """Mean counter values per dispatch, grouped by (kernel, grid size)."""
    rows = list(csv.DictReader(open(path)))
    if not rows:
        print("no rows")
        return
    keys = rows[0].keys()
    kcol = "Kernel_Name" if "Kernel_Name" in keys else "Kernel-Name"
    gcol = "Grid_Size" if "Grid_Size" in keys else ("Grid_Size_X" if "Grid_Size_X" in keys else None)
    dcol = "Dispatch_Id" if "Dispatch_Id" in keys else "Correlation_Id"
    ncol, vcol = "Counter_Name", "Counter_Value"
    acc = defaultdict(lambda: defaultdict(float))
    disp = defaultdict(set)
    for r in rows:
        name = r[kcol]
        if match and match not in name:
            continue
        key = (name, r.get(gcol, "") if gcol else "", r.get("Workgroup_Size", ""))
        acc[key][r[ncol]] += float(r[vcol])
        disp[key].add(r[dcol])
    counters = sorted({c for v in acc.values() for c in v})
    print("mean counter value per dispatch, per kernel and grid size")
    for key in sorted(acc, key=lambda q: -len(disp[q])):
        name, grid, wg = key
        nd = len(disp[key])
        print(f"{name}  grid={grid} workgroup={wg} dispatches={nd}")
        for c in counters:
            if c in acc[key]:
                print(f"    {c:36s} {acc[key][c] / nd:18.1f}")


def summarize_trace(path, match=None, top=40):
    """Per kernel name and grid size: dispatch count and mean, min and max
    duration (microseconds) from rocprofv3's kernel-trace CSV."""
    rows = list(csv.DictReader(open(path)))
    if not rows:
        print("no rows")
        return
    keys = rows[0].keys()
    gcol = "Grid_Size" if "Grid_Size" in keys else "Grid_Size_X"
    acc = defaultdict(list)
    for r in rows:
        name = r["Kernel_Name"]
        if match and match not in name:
            continue
        dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-3
        acc[(name, r.get(gcol, ""), r.get("Workgroup_Size", ""))].append(dur)
    total = sum(sum(v) for v in acc.values())
    print("kernel trace per kernel and grid size (durations in microseconds)")
    print("  calls    total_us    avg_us    min_us    max_us    pct  grid  workgroup  name")
    for key in sorted(acc, key=lambda q: -sum(acc[q]))[:top]:
        v = acc[key]
        name, grid, wg = key
        print(f"{len(v):7d} {sum(v):11.1f} {sum(v) / len(v):9.3f} {min(v):9.3f} {max(v):9.3f} "
              f"{100 * sum(v) / total:6.2f}  {grid} {wg}  {name}")


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", default="poisson3d_q3_32c", choices=sorted(inputs.WORKLOADS))
    r.add_argument("--prec", type=int, default=64, choices=(64, 32))
    r.add_argument("--reps", type=int, default=4)
    r.add_argument("--smooth-only", action="store_true")
    r.add_argument("--nrhs", type=int, default=None, help="right-hand sides (default: the workload's)")
    r.add_argument("--vcycle", action="store_true", help="run V-cycles instead of apply + smoothing step")
    s = sub.add_parser("summarize")
    s.add_argument("csv")
    s.add_argument("--match", default=None)
    t = sub.add_parser("summarize-trace")
    t.add_argument("csv")
    t.add_argument("--match", default=None)
    t.add_argument("--top", type=int, default=40)
    a = ap.parse_args()
    if a.cmd == "run":
        run(a.workload, a.prec, a.reps, a.smooth_only, a.nrhs, a.vcycle)
    elif a.cmd == "summarize":
        summarize(a.csv, a.match)
    else:
        summarize_trace(a.csv, a.match, a.top)


if __name__ == "__main__":
    sys.exit(main())

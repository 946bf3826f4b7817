"""Build libdgmg.so for gfx950 with hipcc: one object per (dimension, degree)
instantiation of the patch kernels, the vector kernels, the host setup and
the C-ABI layer, linked in-tree next to this file.

    python -m paper_2405_18982_amd.build [-j JOBS]
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libdgmg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
DEGREES = range(1, 8)
DIMS = (2, 3)

COMMON = ["-O3", "-std=c++17", "-fPIC", "-fvisibility=hidden", "-I", os.path.join(ROOT, "include")]
# No packed-FP32 instructions in device code (hipcc flag, not a host one).
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _jobs():
    out = []
    src = os.path.join(CSRC, "dgmg_kernels.hip")
    for d in DIMS:
        for k in DEGREES:
            obj = os.path.join(OBJ, f"kernels_d{d}_k{k}.o")
            out.append([HIPCC] + COMMON + DEVICE + [f"-DDGMG_D={d}", f"-DDGMG_K={k}", "-c", src, "-o", obj])
    for name in ("blas", "scratch"):
        out.append([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, f"dgmg_{name}.hip"), "-o",
                                                os.path.join(OBJ, f"{name}.o")])
    for name in ("dgmg_setup", "dgmg_api"):
        out.append([HIPCC] + COMMON + ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include", "-c",
                                        os.path.join(CSRC, name + ".cpp"), "-o",
                                        os.path.join(OBJ, name + ".o")])
    return out


def _run(cmd):
    p = subprocess.run(cmd, capture_output=True, text=True)
    return cmd, p.returncode, p.stdout + p.stderr


def build(jobs=None, verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    cmds = _jobs()
    jobs = jobs or min(16, os.cpu_count() or 4)
    failed = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for cmd, rc, log in ex.map(_run, cmds):
            if rc != 0:
                failed.append((cmd, log))
            elif verbose and log.strip():
                print(log)
    if failed:
        for cmd, log in failed:
            sys.stderr.write(" ".join(cmd) + "\n" + log + "\n")
        raise RuntimeError(f"{len(failed)} compile step(s) failed")
    objs = [c[c.index("-o") + 1] for c in cmds]
    tmp = LIB + ".tmp"
    link = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    cmd, rc, log = _run(link)
    if rc != 0:
        raise RuntimeError("link failed:\n" + log)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("-v", "--verbose", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose))

"""Algorithmic bytes and flops per kernel launch of the SIPG multigrid path,
and the MI355X peaks they are measured against.

Bytes are what one launch must move at minimum (every vector entry it reads
or writes once; cache re-reads of neighbour cells are not counted).  Flops
count the sum-factorised arithmetic of the method as the kernels evaluate it
(cell blocks of the 1-D operators, rank-2 face couplings, tangential masses
of the face data); the fast-diagonalisation solve counts the minimal
2 d n_I^(d+1) multiply-adds of the tensor contractions on the kept space
V_j plus one scaling per kept node.  One multiply-add = 2 flops.
"""

import itertools

PEAK_HBM_GBS = 8000.0          # HBM3E, GB/s
PEAK_FP64_TFLOPS = 78.6        # vector (and matrix) FP64
PEAK_FP32_TFLOPS = 157.3       # vector FP32


def _n_kept(k, N, lo):
    """Dimension of the Dirichlet local space along one direction for the
    patch whose lower cell is `lo` (vertex lo+1)."""
    v = lo + 1
    return 2 * k + int(v == 1) + int(v == N - 1)


def patch_los(N, colour, dim):
    """Lower-cell coordinates along one direction of the patches of a colour."""
    out = []
    for i in range(dim):
        off = (colour >> i) & 1
        cnt = (N - 2) // 2 if off else N // 2
        out.append([off + 2 * m for m in range(cnt)])
    return out


def operator_flops_per_patch(dim, k):
    """Flops of y = A_ref x on one patch tile (all rows), as evaluated."""
    n = k + 1
    E = 2 * n
    sipg = 4 * n * n + 12 * n + 6
    mass = 4 * n * n
    if dim == 3:
        lines = E * E
        passes = (mass + sipg) + (2 * mass + sipg) + (mass + sipg)
        ext_mass = 12 * E * mass          # y-faces along x, z-faces along x and y
        ext_faces = 6 * E * E * (2 * n + 4)
        return lines * passes + ext_mass + ext_faces
    lines = E
    passes = (mass + sipg) + (mass + sipg)
    return lines * passes + 4 * mass + 4 * E * (2 * n + 4)


def apply_counts(dim, k, N, nrhs=1, s=8):
    n = k + 1
    ndof = (N * n) ** dim
    npatch = (N // 2) ** dim
    E = 2 * n
    flops = npatch * (operator_flops_per_patch(dim, k) + E ** dim)
    return dict(bytes=nrhs * 2 * s * ndof, flops=nrhs * flops)


def smooth_colour_counts(dim, k, N, colour, nrhs=1, s=8):
    """One colour launch of the smoother on a level with N cells per direction."""
    n = k + 1
    E = 2 * n
    los = patch_los(N, colour, dim)
    nb = 0
    fl = 0
    for lo in itertools.product(*los):
        nI = [_n_kept(k, N, l) for l in lo]
        vj = 1
        for m in nI:
            vj *= m
        nb += s * (E ** dim + 2 * vj)
        # S_i^T and S_i along each direction: 2 x vj n_I,i multiply-adds; one scaling per node
        fd = 2 * 2 * sum(vj * m for m in nI) + vj
        fl += operator_flops_per_patch(dim, k) + 2 * E ** dim + fd
    return dict(bytes=nrhs * nb, flops=nrhs * fl)


def smooth_step_counts(dim, k, N, nrhs=1, s=8):
    tot = dict(bytes=0, flops=0)
    for c in range(2 ** dim):
        r = smooth_colour_counts(dim, k, N, c, nrhs, s)
        tot["bytes"] += r["bytes"]
        tot["flops"] += r["flops"]
    return tot


def dense_bottom_counts(nd, nrhs=1, s=8):
    """The V-cycle's bottom levels applied as their dense nd x nd operator:
    the matrix read once, b read and x written; one multiply-add per matrix
    entry and right-hand side."""
    return dict(bytes=s * (nd * nd + 2 * nd * nrhs), flops=2 * nd * nd * nrhs)


def bound(counts, seconds, precision=64):
    """Roofline position of a measured launch: achieved GB/s and GFLOP/s, the
    binding resource (larger ideal time) and the fraction of its peak."""
    peak_f = PEAK_FP64_TFLOPS if precision == 64 else PEAK_FP32_TFLOPS
    t_hbm = counts["bytes"] / (PEAK_HBM_GBS * 1e9)
    t_alu = counts["flops"] / (peak_f * 1e12)
    gbs = counts["bytes"] / seconds / 1e9
    tfs = counts["flops"] / seconds / 1e12
    if t_hbm >= t_alu:
        return dict(bound="hbm", achieved=gbs, peak=PEAK_HBM_GBS, unit="GB/s", frac=gbs / PEAK_HBM_GBS,
                    achieved_tflops=tfs, ai=counts["flops"] / counts["bytes"])
    return dict(bound="alu", achieved=tfs, peak=peak_f, unit="TFLOP/s", frac=tfs / peak_f,
                achieved_gbs=gbs, ai=counts["flops"] / counts["bytes"])

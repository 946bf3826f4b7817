"""Host checks of the performance accounting (algorithmic bytes per launch,
roofline classification) and of the benchmark's command-line contract; no
GPU needed."""
import itertools
import os
import subprocess
import sys

import pytest

from paper_2405_18982_amd import roofline

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("dim,k,N", [(2, 1, 8), (2, 3, 16), (3, 2, 8), (3, 3, 4), (3, 7, 8)])
def test_apply_bytes_are_one_read_and_one_write_per_dof(dim, k, N):
    c = roofline.apply_counts(dim, k, N, nrhs=3)
    ndof = 1
    for _ in range(dim):
        ndof *= N * (k + 1)
    assert c["bytes"] == 3 * 2 * 8 * ndof
    assert roofline.apply_counts(dim, k, N, s=4)["bytes"] == 2 * 4 * ndof


@pytest.mark.parametrize("dim,N", [(2, 4), (2, 10), (3, 8), (3, 6)])
def test_colours_cover_every_interior_vertex_once(dim, N):
    seen = set()
    for c in range(2 ** dim):
        for lo in itertools.product(*roofline.patch_los(N, c, dim)):
            v = tuple(l + 1 for l in lo)
            assert all(1 <= vi <= N - 1 for vi in v)
            assert all(((vi + 1) % 2) == ((c >> i) & 1) for i, vi in enumerate(v))
            assert v not in seen
            seen.add(v)
    assert len(seen) == (N - 1) ** dim


def _patches_holding_node_1d(k, N, c, a):
    """Vertex patches whose Dirichlet space holds node a of cell c (1-D): as
    the left cell of vertex c+1 unless a is its left end on an interior face,
    as the right cell of vertex c unless a is its right end on an interior
    face."""
    n = k + 1
    cnt = 0
    if c + 1 <= N - 1 and (a != 0 or c == 0):
        cnt += 1
    if c >= 1 and (a != n - 1 or c == N - 1):
        cnt += 1
    return cnt


@pytest.mark.parametrize("dim,k,N", [(2, 2, 8), (3, 3, 8), (3, 1, 4), (2, 5, 6)])
def test_smoother_bytes_count_vj_by_nodes(dim, k, N):
    """Sum over all colours of the bytes per launch = the tiles read plus b
    and x on V_j; the V_j part must equal the number of (patch, node) pairs
    with the node in the patch's Dirichlet space, counted node by node."""
    s = 8
    E = 2 * (k + 1)
    npatch = (N - 1) ** dim
    tot = roofline.smooth_step_counts(dim, k, N, s=s)["bytes"]
    vj_sum = (tot - s * E ** dim * npatch) // (2 * s)
    per_dir = sum(_patches_holding_node_1d(k, N, c, a) for c in range(N) for a in range(k + 1))
    assert vj_sum == per_dir ** dim


def test_bound_picks_the_slower_resource():
    # 1 GB in 1 ms = 1000 GB/s, far below the ALU time of 1 GFLOP
    r = roofline.bound({"bytes": 1e9, "flops": 1e9}, 1e-3)
    assert r["bound"] == "hbm" and abs(r["achieved"] - 1000.0) < 1e-9
    assert abs(r["frac"] - 1000.0 / roofline.PEAK_HBM_GBS) < 1e-12
    r = roofline.bound({"bytes": 1e6, "flops": 1e12}, 1e-1)
    assert r["bound"] == "alu" and abs(r["achieved"] - 10.0) < 1e-9
    r32 = roofline.bound({"bytes": 1e6, "flops": 1e12}, 1e-1, precision=32)
    assert abs(r32["frac"] - 10.0 / roofline.PEAK_FP32_TFLOPS) < 1e-12


def test_dense_bottom_counts():
    # 3-D Q3: level 1 has 4^3 cells of 4^3 nodes, the operator 4096 x 4096
    nd = 4 ** 3 * 4 ** 3
    c = roofline.dense_bottom_counts(nd)
    assert c["bytes"] == 8 * nd * nd + 16 * nd and c["flops"] == 2 * nd * nd
    assert roofline.bound(c, 20e-6)["bound"] == "hbm"  # 1/4 flop per byte
    c3 = roofline.dense_bottom_counts(nd, nrhs=3, s=4)
    assert c3["bytes"] == 4 * (nd * nd + 6 * nd) and c3["flops"] == 6 * nd * nd


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr and p.stdout.strip() == ""

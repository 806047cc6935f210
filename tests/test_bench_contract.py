"""bench.py's host-side contract, without a GPU: the algorithmic bytes and flops it prices the
roofline with (pinned to the per-product totals of the 16^3 p = 8 and 8^3 p = 16 workloads and
to the per-DOF figures of the stored-factor product), the traffic it reads from the committed
counter summary, and its refusal of more than one GPU."""

import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_and_flops_of_the_workloads():
    n3 = 16 * 8 + 1
    N = n3 ** 3
    assert N == 2146689
    # 16^3 hexes at p = 8: 6 factors per point, x and y once (FP64)
    assert bench.apply_bytes(3, (16, 16, 16), 8, N, 8) == 8 * (6 * 4096 * 729 + 2 * N) == 177674256
    assert bench.apply_bytes(3, (16, 16, 16), 8, N, 4) == 177674256 // 2
    assert bench.apply_flops(3, (16, 16, 16), 8) == 4096 * (12 * 9 ** 4 + 15 * 9 ** 3) == 367276032
    # 8^3 hexes at p = 16: the same node count
    assert bench.apply_bytes(3, (8, 8, 8), 16, N, 8) == 8 * (6 * 512 * 17 ** 3 + 2 * N) == 155088912
    assert bench.apply_flops(3, (8, 8, 8), 16) == 512 * (12 * 17 ** 4 + 15 * 17 ** 3)
    # 2D: 3 factors per point
    n2 = 512 * 8 + 1
    assert bench.apply_bytes(2, (512, 512), 8, n2 * n2, 8) == 8 * (3 * 512 * 512 * 81 + 2 * n2 * n2)


@pytest.mark.parametrize("p,bytes_per_dof", [(4, 109.8), (8, 84.3), (16, 73.6)])
def test_bytes_per_dof_of_large_meshes(p, bytes_per_dof):
    """Per DOF on a large 3D mesh (the boundary's share negligible): 8 (6 n^3 / p^3 + 2) bytes."""
    ne = 48
    N = (ne * p + 1) ** 3
    b = bench.apply_bytes(3, (ne, ne, ne), p, N, 8) / N
    assert abs(b - bytes_per_dof) < 0.02 * bytes_per_dof


def test_traffic_is_read_only_for_its_problem():
    t = bench.measured_traffic(16, 8)
    if t is not None:  # present while the summary's source hash matches the apply kernels
        assert 177674256 <= t <= 2 * 177674256
    assert bench.measured_traffic(8, 16) is None
    assert bench.measured_traffic(32, 8) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""

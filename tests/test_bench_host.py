"""Host-side parts of the benchmark contract (no GPU): the one-GPU guard, and
the algorithmic byte counts' dependence on the work they describe."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1805_04155_amd import workloads as W  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _bytes(listed, plastic_elems, plastic_ips, tangent_bytes=8):
    wl = W.workload_p1_square(8)
    counts = {"plastic_elems": plastic_elems, "plastic_ips": plastic_ips, "listed": listed,
              "n_perm": wl.mesh.n_elems}
    return wl.mesh, bench.kernel_bytes(wl.mesh, wl.material, counts, tangent_bytes)


def test_assembly_bytes_scale_with_the_work_list():
    mesh, b0 = _bytes(0, 0, 0)
    _, b1 = _bytes(10, 10, 10)
    _, b2 = _bytes(20, 20, 20)
    assert b0["assembly"] == 0
    assert b2["assembly"] == 2 * b1["assembly"]
    # per listed element at least its n_p^2 node blocks, read and written
    blk = mesh.n_p ** 2 * 2 * mesh.dim ** 2 * 8
    assert b1["assembly"] >= 10 * blk
    # FP32 tangent values halve the value bytes only
    _, b1f = _bytes(10, 10, 10, tangent_bytes=4)
    assert b1["assembly"] - b1f["assembly"] == 10 * mesh.n_p ** 2 * 2 * mesh.dim ** 2 * 4



def test_scalar_model_bytes_of_the_headline_pass():
    """The scalar-CSR byte model on the 64^3 cube at half of the elements
    plastic: 1048576 plastic points at 8 (24 + 1) + 64 = 264 B and 131072
    plastic elements at 576 x (4 + 16) x 2 = 23040 B (FP64)."""
    mesh = W.mesh_q1_3d(2, 2, 2, 1.0, 1.0, 1.0)
    counts = {"plastic_elems": 131072, "plastic_ips": 1048576}
    assert bench.assembly_bytes_scalar_model(mesh, counts, 8) == \
        1048576 * 264 + 131072 * 23040
    assert bench.assembly_bytes_scalar_model(mesh, counts, 4) == \
        1048576 * 264 + 131072 * 576 * 12 * 2

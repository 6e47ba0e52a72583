"""Host-side parts of bench.py (no GPU): the algorithmic byte count the
roofline divides by, and the one-GPU contract."""
import os
import subprocess
import sys

import numpy as np

import rlb_inputs as ri

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_sphere_algorithmic_bytes_from_an_independent_count():
    """200x100x100 sphere: solid cells are the integer points with
    (x-60)^2 + (y-50)^2 + (z-50)^2 <= 15^2, counted here by brute force; the
    x = 0 plane is the inflow plane (no solid on it).  Every other cell reads
    and writes 2 x 19 FP64 values, inflow cells write them only, and every
    cell reads its 4-byte cell word."""
    x, y, z = np.meshgrid(np.arange(200), np.arange(100), np.arange(100), indexing="ij")
    solid = int(((x - 60) ** 2 + (y - 50) ** 2 + (z - 50) ** 2 <= 15 ** 2).sum())
    inflow = 100 * 100
    cells = 200 * 100 * 100
    upd = cells - solid - inflow
    want = upd * 2 * 19 * 2 * 8 + inflow * 2 * 19 * 8 + 4 * cells
    got = bench.algorithmic_bytes(ri.sphere(), 8)
    assert got["solid_cells"] == solid
    assert got["inflow_cells"] == inflow
    assert got["updated_cells"] == upd
    assert got["bytes"] == want
    assert got["bytes_per_updated_cell"] == 608


def test_periodic_box_bytes_have_no_class_bytes():
    s = ri.random_state_setup(8, 8, 8, seed=1)
    got = bench.algorithmic_bytes(s, 4)
    assert got["bytes"] == 512 * 2 * 19 * 2 * 4 and got["inflow_cells"] == 0


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

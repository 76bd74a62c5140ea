"""Host-side checks of bench.py (no GPU)."""
import os
import subprocess
import sys

import numpy as np
import pytest

from oracle import fem, qtt, tt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


@pytest.mark.parametrize("level", [2, 3, 4])
def test_closed_form_field_tt_equals_nodal_field(level):
    c = [0.7, -1.3, 0.2]
    full = tt.tt_full(bench.manufactured_field_cores(level, c)).reshape(-1)
    g = fem.Grid(3, level)
    ref = qtt.to_qtt_order(fem.manufactured_u(g.node_coords(), c).reshape(-1), 3, level)
    assert np.abs(full - ref).max() <= 1e-14 * np.abs(ref).max()


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr

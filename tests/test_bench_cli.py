"""bench.py without a GPU: the one-GPU contract and the algorithmic-byte
arithmetic its roofline figures use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes():
    t = {"window_edges": 10, "arcs": 3, "touched_nodes": 5, "touched_edges": 7, "sweep_ms": 2.0}
    # 12 B per window edge, 32 B per arc (written and read back), (2 + c) x 8 B
    # per touched node, 8 B per touched edge
    assert bench.algorithmic_bytes(t, 25) == 12 * 10 + 32 * 3 + 8 * 27 * 5 + 8 * 7
    frac = bench.hbm_frac(t, 25)
    assert abs(frac - bench.algorithmic_bytes(t, 25) / 2e-3 / 1e9 / 8000.0) < 1e-15
    assert bench.hbm_frac(dict(t, sweep_ms=0.0), 25) is None

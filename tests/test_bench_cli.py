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


def test_traffic_entries_match_launches():
    """A profiled traffic figure is reported only for the kernel source it was
    taken on and the exact launch (grid, hubs, own arc buffer, pairs): an
    entry taken on another source of the kernel matches nothing."""
    sha = bench.sha256(bench.SWEEP_SRC)
    for workload, entries in bench.TRAFFIC.items():
        assert entries, workload
        for tr in entries:
            launch = {"n_slabs": tr["slabs"], "hub_nodes": tr["hub_nodes"], "arc_cap": tr["arc_cap"]}
            want = tr if tr["sweep_sha256"] == sha else None
            assert bench.traffic_of(workload, launch, tr["pairs_per_launch"]) is want
            for key, bad in (("n_slabs", tr["slabs"] + 1), ("hub_nodes", tr["hub_nodes"] + 1),
                             ("arc_cap", tr["arc_cap"] - 1)):
                assert bench.traffic_of(workload, dict(launch, **{key: bad}), tr["pairs_per_launch"]) is None
            assert bench.traffic_of(workload, launch, tr["pairs_per_launch"] + 1) is None
    assert bench.traffic_of("no-such-workload", {"n_slabs": 1, "hub_nodes": 0, "arc_cap": 1}, 1) is None
    r = bench.roofline({"sweep_ms": 2.0, "launches": 1, "window_edges": 10, "arcs": 0, "touched_nodes": 0,
                        "touched_edges": 0}, "no-such-workload", {"n_slabs": 1, "hub_nodes": 0, "arc_cap": 1},
                       "k", 1)
    assert r["traffic"] is None and r["traffic_slabs"] is None and abs(r["frac"] - 120 / 2e-3 / 1e9 / 8000.0) < 1e-15

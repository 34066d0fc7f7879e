"""Host-side checks of bench.py: the one-GPU contract, the flop count behind the throughput, and
the committed rocprofv3 summary that supplies the roofline object's traffic figure."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    # the check runs before torch is imported, so this touches no device
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert r.stdout == ""
    assert "single MI355X" in r.stderr


def _count_pass_flops(m, n):
    """Operation count of one Cholesky QR pass written out as loops: the upper triangle of
    X^T X (one multiply and one add per term), then the row-wise triangular solve Q = X R^{-1}
    (per row: n divisions and, for each pair k < j, one multiply and one subtract)."""
    ops = 0
    for i in range(n):
        for j in range(i, n):
            ops += 2 * m
    for _ in range(m):
        for j in range(n):
            ops += 1 + 2 * j
    return ops


def test_flop_count_matches_loops():
    for m, n, p in [(7, 1, 1), (10, 3, 2), (33, 8, 5), (5, 16, 3)]:
        assert bench.flops_of(m, n, p) == p * _count_pass_flops(m, n)


def test_committed_profile_is_consistent():
    for w in ["c2"]:
        path = os.path.join(ROOT, "profiles", f"trsm_gram_{w}_counters.json")
        with open(path) as fh:
            c = json.load(fh)
        m, n = bench.WORKLOADS[w][:2]
        assert c["algorithmic_bytes_per_launch"] == 16 * m * n
        ratio = c["hbm_bytes_per_launch"] / c["algorithmic_bytes_per_launch"]
        assert 1.0 <= ratio < 1.5
        # the traffic figure is reported only while the kernel sources are those profiled
        got = bench.traffic_from_profiles("trsm_gram", w, 0)
        if c["source_hash"] == bench.source_hash():
            assert got == c["hbm_bytes_per_launch"]
        else:
            assert got is None
        # every command of the summary runs committed files only
        for cmd in c["commands"].values():
            assert "_work" not in cmd
            assert "bench.py" in cmd
        with open(os.path.join(ROOT, "profiles", f"trsm_gram_{w}.md")) as fh:
            md = fh.read()
        assert c["source_hash"] in md

"""The committed HBM counter summary belongs to the current kernel sources
(otherwise bench.py reports roofline.traffic as null)."""
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_hbm_summary_matches_kernel_sources():
    import bench
    with open(bench.TRAFFIC_FILE) as f:
        m = re.search(r"kernel_source_sha256: ([0-9a-f]{64})", f.read())
    assert m, "no kernel hash in the counter summary"
    assert m.group(1) == bench.kernel_source_hash(), "kernel sources changed since the HBM counters were taken"
    assert bench.measured_traffic("multi_colloid256") is not None

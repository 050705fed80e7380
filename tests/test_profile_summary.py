"""The committed HBM counter summaries belong to the current kernel sources
(otherwise bench.py reports roofline.traffic as null)."""
import glob
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_hbm_summaries_match_kernel_sources():
    import bench
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "k_march_fire_*_hbm.txt")))
    assert bench.TRAFFIC_FILE in files
    for path in files:
        vals = bench.read_summary(path)
        m = re.fullmatch(r"k_march_fire_(f32|f64)_(\w+?)_hbm\.txt", os.path.basename(path))
        assert m, path
        assert vals.get("workload") == m.group(2), path
        assert vals.get("kernel_source_sha256") == bench.kernel_source_hash(), \
            f"kernel sources changed since the HBM counters of {os.path.basename(path)} were taken"
        assert bench.measured_traffic(m.group(2), m.group(1)) is not None

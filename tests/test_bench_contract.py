"""Host-side parts of the benchmark contract (no GPU needed)."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_hash_and_workloads():
    import bench
    assert re.fullmatch(r"[0-9a-f]{64}", bench.kernel_source_hash())
    for name in ("multi_colloid256", "bulk256", "bulk256_f64", "bulk256_l23", "colloid_slab128",
                 "colloid_slab128_f32", "patterned_wall512", "bulk32"):
        cfg = bench.workload(name)
        d = bench.describe(cfg)
        assert d["workload"] == cfg["name"] and d["state_dtype"] in ("f32", "f64")
    assert bench.workload("multi_colloid256")["shape"] == (256, 256, 256)
    assert bench.workload("patterned_wall512")["prec"] == "f32"
    # the counter summary covers the headline workload only
    assert bench.measured_traffic("multi_colloid256") is not None
    assert bench.measured_traffic("bulk256") is None

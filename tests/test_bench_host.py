"""Host-side behaviour of bench.py that needs no GPU: the one-GPU rule and
the source hash that gates the committed HBM-traffic figures."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def test_traffic_figures_follow_the_sources():
    import bench

    h = bench.kernel_source_hash()
    assert len(h) == 64
    if not os.path.exists(bench.TRAFFIC_FILE):
        # no committed counter summary for the workload: no traffic figure
        assert bench.measured_traffic("spmv_proj") is None
        return
    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    for k in ("spmv_proj", "update_proj", "update_norm"):
        assert k in t["kernels"]
        assert t["kernels"][k]["traffic_bytes_per_launch"] > 0
    if t["source_sha256"] == h:
        assert bench.measured_traffic("spmv_proj") == t["kernels"]["spmv_proj"]["traffic_bytes_per_launch"]
    else:
        assert bench.measured_traffic("spmv_proj") is None

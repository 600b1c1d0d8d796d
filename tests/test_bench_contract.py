"""bench.py's command-line contract on the CPU: one GPU only, and the format
of the committed counter summary it reads the sweep's HBM traffic from."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, env={**os.environ, "WORLD_SIZE": "1"})
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_traffic_summary_format():
    """The committed counter summary carries the bytes per launch and the
    digest of the sweep source it was measured on (bench.py reports null
    traffic whenever that digest differs from the current source)."""
    sys.path.insert(0, ROOT)
    import bench
    vals = {}
    with open(os.path.join(ROOT, "profiles", "k_sweep_interface3d_128_traffic.md")) as f:
        for line in f:
            if line.startswith("traffic:"):
                vals = dict(kv.split("=") for kv in line.split()[1:])
    assert float(vals["bytes_per_launch"]) > 0 and float(vals["fetch"]) > 0 and float(vals["write"]) > 0
    assert len(vals["source"]) == len(bench.kernel_source_digest()) == 16

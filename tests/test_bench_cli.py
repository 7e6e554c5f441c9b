"""bench.py's command line without a GPU: more than one GPU is refused with a
message, and the roofline helper reads the committed counter summary only
for the kernel source it was taken on."""
import hashlib
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_read_for_the_recorded_kernel_source_only():
    sys.path.insert(0, ROOT)
    import bench
    t = json.load(open(bench.TRAFFIC_FILE))
    sha = hashlib.sha256(open(bench.KERNEL_SRC, "rb").read()).hexdigest()
    k = "alks_step_kernel<float, false, 4>"
    got = bench.traffic_per_launch(k)
    if t["source_sha256"] == sha:
        d = t["kernels"][k]
        assert got == d["fetch_kib"] * 1024 / t["fetch_factor"] + d["write_kib"] * 1024 / t["write_factor"]
    else:
        assert got is None
    assert bench.traffic_per_launch("no_such_kernel") is None

"""bench.py's command line without a GPU: more than one GPU is refused with a
message, the roofline helper takes the algorithmic bytes per update and
reads the committed counter summary only for the kernel sources it was taken
on."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_is_read_for_the_recorded_kernel_sources_only(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    sha = bench.sources_sha()
    rec = {"source_sha256": sha, "fetch_factor": 0.5, "write_factor": 1.0,
           "entries": {"headline|k<float>": {"fetch_kib": 10.0, "write_kib": 4.0}}}
    f = tmp_path / "t.json"
    f.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.traffic_per_launch("headline", "k<float>") == 10.0 * 1024 / 0.5 + 4.0 * 1024
    assert bench.traffic_per_launch("batch", "k<float>") is None
    assert bench.traffic_per_launch("headline", "no_such_kernel") is None
    rec["source_sha256"] = dict(sha, **{"lks_kernels.hip": "0" * 64})
    f.write_text(json.dumps(rec))
    assert bench.traffic_per_launch("headline", "k<float>") is None


def test_roofline_uses_the_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    r = bench.roofline("nowhere", "k", ("2d", "adj_steady"), "float", 524288, 10.0)
    assert r["bytes_per_node_update"] == 60
    assert r["achieved"] == pytest.approx(60 * 524288 / 10e-6 / 1e9, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-12)
    assert r["library_bytes_per_node_update"] == 37
    r64 = bench.roofline("nowhere", "k", ("3d_thermal", "adj_unsteady"), "double", 10, 1.0)
    assert r64["bytes_per_node_update"] == 280


def test_bench_options_parse():
    sys.path.insert(0, ROOT)
    import bench
    a = bench.parse(["--only", "headline,batch", "--shapes", '{"batch": {"fp32": [16, 1, 1]}}'])
    assert a.only == "headline,batch"
    assert json.loads(a.shapes)["batch"]["fp32"] == [16, 1, 1]

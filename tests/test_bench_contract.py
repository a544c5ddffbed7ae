"""bench.py behaviour that needs no GPU."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stdout


def test_traffic_record_requires_matching_source_and_options():
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "k_hs_fp64_traffic.json")))
    opts = rec.get("options", {"waves": 4, "tile_group": 0})
    import hashlib
    srcs = rec["source"] if isinstance(rec["source"], list) else [rec["source"]]
    sha = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in srcs)).hexdigest()[:16]
    got = bench.recorded_traffic(rec["workload"], opts)
    if sha == rec["source_sha256_16"]:
        assert got == rec["traffic_bytes"]
    else:
        assert got is None
    assert bench.recorded_traffic("another-workload", opts) is None
    assert bench.recorded_traffic(rec["workload"], {"waves": 99, "tile_group": 99}) is None

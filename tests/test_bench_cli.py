"""The benchmark's command-line contract, checked on the host: more than one
GPU is refused with a message before any device work, and the source digests
that key the committed counter records are stable."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "GPU" in (r.stdout + r.stderr)


def test_traffic_record_names_the_current_gemm_source():
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    for key, r in rec.items():
        assert r["hbm_bytes_per_launch"] > 0 and r["kernel"]
        # a record whose digest no longer matches is ignored by the bench (traffic null)
        got = bench.traffic_for(key, r["kernel"].split("<")[0], r["source_digest"])
        assert got == r["hbm_bytes_per_launch"]
    assert bench.traffic_for("sq4096_b36", "int8_digits_gemm_kernel", "0" * 16) is None

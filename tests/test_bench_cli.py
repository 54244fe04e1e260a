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


def test_binding_roof():
    # the headline (8192^3, (2,2) words) is bound by the FP64 matrix cores;
    # the tall-skinny 16384^2 x 256 product at three digits by HBM: its 2.17
    # GB of planes and C take 0.272 ms at 8 TB/s, its 1.24e12 digit-product
    # operations 0.247 ms at 5 POP/s
    sys.path.insert(0, ROOT)
    import bench
    fp = {"form": 1, "digits_a": 0, "digits_b": 0}
    work = 2.0 * 4 * 8192.0 ** 3
    r = bench.binding_roof(fp, 8192, 8192, 8192, work, bench.FP64_MFMA_PEAK_TFLOPS, "TFLOP/s", 100.0)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert abs(r["frac"] - work / 0.1 / 78.6e12) < 1e-4
    i8 = {"form": 2, "digits_a": 3, "digits_b": 3}
    work = 2.0 * 9 * 16384.0 ** 2 * 256
    r = bench.binding_roof(i8, 16384, 16384, 256, work, bench.INT8_MFMA_PEAK_TOPS, "TOP/s", 0.644)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    alg = 3 * 16384 * 256 * 2 + 8 * 16384 ** 2
    assert r["algorithmic_bytes_per_launch"] == alg
    assert abs(r["achieved"] - alg / 0.644e-3 / 1e9) < 1e-2
    # seven digits: the digit products bind again
    i8 = {"form": 2, "digits_a": 7, "digits_b": 7}
    work = 2.0 * 49 * 16384.0 ** 2 * 256
    assert bench.binding_roof(i8, 16384, 16384, 256, work, bench.INT8_MFMA_PEAK_TOPS, "TOP/s", 2.45)["bound"] == "mfma"

"""Host-side parts of bench.py's result line, checked without a GPU:

* a request for more than one GPU exits with a message (one-GPU path only);
* the recorded HBM traffic of the substitution kernel is reported only while
  the kernel source matches the one the counters were taken with;
* the CPU baseline leg times the oracle on a bounded sample and reports the
  fields of the contract (value, unit, cores, kind, sample).
"""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_recorded_traffic_gated_by_kernel_source(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "k_solve_chain2_2d1024_traffic.json")) as fh:
        rec = json.load(fh)
    got = bench.recorded_traffic("chain2")
    assert got is None or got == rec["traffic_bytes_per_launch"]
    # a traffic record is never older than the algorithmic bytes it should cover
    assert rec["traffic_bytes_per_launch"] >= 10.933e9
    assert bench.recorded_traffic("perline") is None       # no record for that kernel

    import hashlib

    class _H:
        def __init__(self, *a):
            pass

        def hexdigest(self):
            return "0" * 64
    monkeypatch.setattr(hashlib, "sha256", _H)
    assert bench.recorded_traffic("chain2") is None


def test_cpu_baseline_fields():
    cb = bench.run_cpu_baseline(4, 64, 19, 1e-6)
    assert cb["value"] > 0 and cb["unit"] == "solves/s"
    assert cb["kind"] == "oracle" and cb["cores"] >= 1
    assert "oracle" in cb["sample"] and "4x4" in cb["sample"]

"""Host-side parts of bench.py's result line, checked without a GPU:

* a request for more than one GPU exits with a message (one-GPU path only);
* the HBM traffic record is built from the two counter runs (FETCH_SIZE and
  WRITE_SIZE per dispatch, each scaled by what it reads for the 1 GiB copy)
  and reported only while the kernel source matches the one the counters
  were taken with;
* the CPU baseline legs time the oracle on a bounded sample and report the
  fields of the contract (value, unit, cores, kind, sample).
"""
import csv
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


def _counter_csv(d, counter, rows):
    os.makedirs(os.path.join(d, "host"), exist_ok=True)
    with open(os.path.join(d, "host", "123_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for did, name, v in rows:
            wr.writerow([did, name, counter, v])


def test_traffic_record_from_counter_runs(tmp_path, monkeypatch):
    k = "void ddm::k_solve_mma<HIP_vector_type<float, 2u>, 768>(...)"
    cp = "void at::native::elementwise_kernel<copy...>"
    # FETCH_SIZE reads half the bytes of the copy, WRITE_SIZE all of them
    _counter_csv(str(tmp_path / "f"), "FETCH_SIZE", [(1, "fill", 10.0), (2, k, 1000.0), (3, k, 1002.0),
                                                      (4, k, 998.0), (5, cp, 524288.0)])
    _counter_csv(str(tmp_path / "w"), "WRITE_SIZE", [(1, "fill", 10.0), (2, k, 100.0), (3, k, 100.0),
                                                      (4, k, 100.0), (5, cp, 1048576.0)])
    prof = tmp_path / "profiles"
    prof.mkdir()
    bench.make_traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), "test_c64", variant="mma",
                              profiles_dir=str(prof))
    with open(prof / "k_solve_mma_test_c64_traffic.json") as fh:
        rec = json.load(fh)
    assert abs(rec["fetch_bytes_per_launch"] - 1000.0 * 1024 * 2) < 1e-6
    assert abs(rec["write_bytes_per_launch"] - 100.0 * 1024) < 1e-6
    assert rec["traffic_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    got = bench.recorded_traffic("mma", "test_c64", profiles_dir=str(prof))
    assert got == rec["traffic_bytes_per_launch"]
    assert bench.recorded_traffic("perline", "test_c64", profiles_dir=str(prof)) is None  # no record
    # a changed kernel source voids the record
    monkeypatch.setattr(bench, "kernel_sha", lambda v: "0" * 64)
    assert bench.recorded_traffic("mma", "test_c64", profiles_dir=str(prof)) is None


def test_committed_traffic_record_covers_algorithmic_bytes():
    path = os.path.join(ROOT, "profiles", "k_solve_mma_layered2048_c64_traffic.json")
    if not os.path.exists(path):
        return
    with open(path) as fh:
        rec = json.load(fh)
    # every complex64 inverse of the 2048^2 layered workload read once per sweep: 24.3 GB
    assert rec["fetch_bytes_per_launch"] >= 24.0e9


def test_cpu_baseline_fields():
    cb = bench.run_cpu_baseline(4, 64, 19, 1e-6)
    assert cb["value"] > 0 and cb["unit"] == "solves/s"
    assert cb["kind"] == "oracle" and cb["cores"] >= 1
    assert "oracle" in cb["sample"] and "4x4" in cb["sample"]


def test_cpu_baseline_layered_fields():
    cb = bench.run_cpu_baseline_layered(16, 256, 256)
    assert cb["value"] > 0 and cb["unit"] == "solves/s"
    assert cb["kind"] == "oracle" and cb["cores"] >= 1
    assert "layered 2048^2" in cb["sample"] and "4x4" in cb["sample"]


def test_overlap_report_on_a_synthetic_trace(tmp_path):
    """Two streams: a substitution kernel [0, 100) on stream 1, a transfer
    [50, 150) on stream 2, a residual [200, 300) on stream 1 alone."""
    path = tmp_path / "trace.csv"
    with open(path, "w", newline="") as fh:
        wr = csv.writer(fh)
        wr.writerow(["Kind", "Stream_Id", "Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        wr.writerow(["KERNEL_DISPATCH", 1, "void ddm::k_solve_mma<float>", 0, 100])
        wr.writerow(["KERNEL_DISPATCH", 2, "void ddm::k_transfer<float>", 50, 150])
        wr.writerow(["KERNEL_DISPATCH", 1, "void ddm::k_stencil<0>", 200, 300])
    rep = bench.overlap_report(str(path))
    assert rep["kernels"] == 3 and rep["streams"] == 2
    assert abs(rep["busy_ms"] - 250e-6) < 1e-12 and abs(rep["multi_stream_ms"] - 50e-6) < 1e-12
    assert abs(rep["overlapped_share_by_class"]["substitution"] - 0.5) < 1e-12
    assert abs(rep["overlapped_share_by_class"]["transfer"] - 0.5) < 1e-12
    assert rep["overlapped_share_by_class"]["residual"] == 0.0


def test_traffic_lookups_name_committed_records():
    """Every traffic record bench.py looks up (the tag of each
    recorded_traffic call, with the variant its workload runs) is a committed
    file under profiles/: a lookup under another tag would report no
    traffic even with the counters taken."""
    import re
    with open(os.path.join(ROOT, "bench.py")) as fh:
        tags = set(re.findall(r'recorded_traffic\([^,]+,\s*"([^"]+)"\)', fh.read()))
    assert tags == {"layered2048_c64", "2d1024"}
    for variant, tag in (("mma", "layered2048_c64"), ("chain2", "2d1024")):
        path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (bench.SUBST_KERNELS[variant], tag))
        assert os.path.exists(path), path

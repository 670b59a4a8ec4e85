"""Host logic of bench.py that needs no GPU: the one-GPU refusal, the
calibration of the HBM traffic counters against the copy kernel, and the
rule that a stored traffic figure is reported only while the kernel sources
it was measured on are unchanged."""
import csv
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""  # no JSON line


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_calibrated_by_the_copy_kernel(tmp_path, monkeypatch):
    out = tmp_path / "traffic.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    part = "void pic::k_particles<3, float, 1024, 0>(pic::BatchTable const*)"
    copy = "pic::k_copy_bench(void const*, void*, long)"
    kib = bench.COPY_BYTES / 1024.0
    # the copy reads and writes COPY_BYTES; FETCH_SIZE counts half its bytes
    # (as measured on the device), WRITE_SIZE all of them
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    _counter_csv(fetch, "FETCH_SIZE", [(copy, kib / 2), (copy, kib / 2), (part, 1000.0), (part, 3000.0)])
    _counter_csv(write, "WRITE_SIZE", [(copy, kib), (part, 4000.0), (part, 4000.0)])
    bench.summarize_traffic(str(fetch), str(write), "c5", ["cmd a", "cmd b"])
    kv = {}
    for line in out.read_text().splitlines():
        if line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    # particle kernel: mean 2000 KiB fetched x 2, 4000 KiB written x 1
    assert float(kv["fetch_scale"]) == pytest.approx(2.0)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    assert float(kv["fetch_bytes_per_launch"]) == pytest.approx(2000 * 1024 * 2, rel=1e-4)
    assert float(kv["write_bytes_per_launch"]) == pytest.approx(4000 * 1024, rel=1e-4)
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx((4000 + 4000) * 1024, rel=1e-6)
    assert kv["dispatches_fetch"] == "2" and kv["dispatches_write"] == "2"
    # reported for this workload while the sources hash the same, else not
    assert bench.read_traffic("c5") == pytest.approx(8000 * 1024)
    assert bench.read_traffic("c3") is None
    text = out.read_text().replace(bench.kernel_source_hash(), "0" * 64)
    out.write_text(text)
    assert bench.read_traffic("c5") is None


"""The measured-traffic records of bench.py: HBM bytes per launch from two
rocprofv3 counter files (FETCH_SIZE, WRITE_SIZE), each counter scaled by what
it reads for the plain 1 GiB copy of the same run; one record per kernel,
read back only while the kernel sources hash to the stored value.  Host logic
on synthetic counter files (no GPU)."""

import csv
import json

import pytest

import bench

KIB = 1 << 30 >> 10          # a 1 GiB copy in KiB


def _counter_file(path, counter, copy_kib, kernels):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for v in copy_kib:
            w.writerow({"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": counter, "Counter_Value": v})
        for name, vals in kernels.items():
            for v in vals:
                w.writerow({"Kernel_Name": f"void {name}(int, double*)", "Counter_Name": counter, "Counter_Value": v})
        w.writerow({"Kernel_Name": "void other()", "Counter_Name": "SQ_WAVES", "Counter_Value": 1})
    return str(path)


@pytest.fixture
def traffic_file(tmp_path, monkeypatch):
    path = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    return path


def test_scaled_bytes_and_lookup(tmp_path, traffic_file):
    k64 = bench.STENCIL[(True, "fp64")]
    # FETCH_SIZE reads half of the copy's 2^30 bytes (scale 2), WRITE_SIZE all of it;
    # small copies (below 90% of the largest) are not calibration copies
    f = _counter_file(tmp_path / "f.csv", "FETCH_SIZE", [KIB / 2, KIB / 2, 100.0], {k64: [1000.0, 3000.0]})
    w = _counter_file(tmp_path / "w.csv", "WRITE_SIZE", [KIB, KIB], {k64: [500.0, 500.0]})
    bench.write_traffic(f, w, k64, "cmd")
    t = json.load(open(traffic_file))["records"]
    assert len(t) == 1 and t[0]["kernel"] == k64 and t[0]["launches"] == [2, 2]
    assert t[0]["fetch_scale"] == pytest.approx(2.0) and t[0]["write_scale"] == pytest.approx(1.0)
    assert bench.measured_traffic(k64) == pytest.approx(1024.0 * (2000.0 * 2.0 + 500.0))
    assert bench.measured_traffic(bench.STENCIL[(True, "fp32")]) is None


def test_one_record_per_kernel_and_stale_records(tmp_path, traffic_file, monkeypatch):
    k64, k32 = bench.STENCIL[(True, "fp64")], bench.STENCIL[(True, "fp32")]
    f = _counter_file(tmp_path / "f.csv", "FETCH_SIZE", [KIB / 2], {k64: [10.0], k32: [4.0]})
    w = _counter_file(tmp_path / "w.csv", "WRITE_SIZE", [KIB], {k64: [1.0], k32: [1.0]})
    bench.write_traffic(f, w, k64, "cmd")
    bench.write_traffic(f, w, k32, "cmd")
    bench.write_traffic(f, w, k64, "cmd")            # replaces, does not duplicate
    kernels = [r["kernel"] for r in json.load(open(traffic_file))["records"]]
    assert sorted(kernels) == sorted([k64, k32])
    assert bench.measured_traffic(k32) == pytest.approx(1024.0 * (8.0 + 1.0))
    # once the kernel sources change, no record is read, and a new record drops the stale ones
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "changed")
    assert bench.measured_traffic(k64) is None and bench.measured_traffic(k32) is None
    bench.write_traffic(f, w, k64, "cmd")
    assert [r["kernel"] for r in json.load(open(traffic_file))["records"]] == [k64]


def test_missing_rows_are_an_error(tmp_path, traffic_file):
    k64 = bench.STENCIL[(True, "fp64")]
    f = _counter_file(tmp_path / "f.csv", "FETCH_SIZE", [], {k64: [1.0]})
    w = _counter_file(tmp_path / "w.csv", "WRITE_SIZE", [KIB], {k64: [1.0]})
    with pytest.raises(SystemExit):
        bench.write_traffic(f, w, k64, "cmd")


def test_committed_record_reads_back():
    """The committed record holds both dominant kernels of the 32^4 workload."""
    recs = bench.traffic_records()
    assert {r["kernel"] for r in recs} >= {bench.STENCIL[(True, "fp64")], bench.STENCIL[(True, "fp32")]}
    for r in recs:
        assert r["traffic_bytes_per_launch"] > 1e9 and r["command"].startswith("rocprofv3 --pmc")

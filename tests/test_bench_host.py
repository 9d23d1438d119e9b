"""Host logic of bench.py (CPU): the HBM-traffic summary built from two
rocprofv3 counter runs, scaled by the calibration copy of known size."""
import csv
import json
import os

import pytest

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for did, kernel, value in rows:
            w.writerow({"Dispatch_Id": did, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_summarize_pmc_scales_by_the_calibration_copy(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    prod = "void lsdm::k_gprod_rs<float, false>(...)"
    # the fetch counter reads half of the 1 GiB copy (split over two XCD rows),
    # the write counter all of it; a non-product kernel is left out
    _write(tmp_path / "f", "FETCH_SIZE", [(1, copy, 262144.0), (1, copy, 262144.0), (2, prod, 1000.0),
                                          (3, "void lsdm::k_sym_fill<float>(...)", 50.0), (4, prod, 10.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(1, copy, 1048576.0), (2, prod, 200.0), (4, prod, 0.0)])
    out = tmp_path / "t.json"
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "fp32", str(out))
    t = json.loads(out.read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["kernel_hash"] == bench.kernel_hash() and t["prec"] == "fp32"
    assert [d["id"] for d in t["dispatches"]] == [2, 4]
    assert t["dispatches"][0]["fetch_bytes"] == pytest.approx(1000.0 * 2.0 * 1024)
    assert t["dispatches"][0]["write_bytes"] == pytest.approx(200.0 * 1024)


def test_summarize_pmc_needs_the_calibration_copy(tmp_path):
    prod = "void lsdm::k_gprod_rs<float, false>(...)"
    _write(tmp_path / "f", "FETCH_SIZE", [(2, prod, 1000.0)])
    _write(tmp_path / "w", "WRITE_SIZE", [(2, prod, 200.0)])
    with pytest.raises(SystemExit):
        bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), "fp32", str(tmp_path / "t.json"))


def test_traffic_reported_only_for_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    summ = {"kernel_hash": bench.kernel_hash(), "prec": "fp32", "steps": 1,
            "dispatches": [{"fetch_bytes": 3.0e9, "write_bytes": 1.0e9}, {"fetch_bytes": 2.0e9, "write_bytes": 0.5e9}]}
    f.write_text(json.dumps(summ))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    wl = bench.DEFAULT_WORKLOAD
    assert bench.traffic_per_step("fp32", wl) == pytest.approx(6.5e9)
    assert bench.traffic_per_step("fp64", wl) is None                  # another precision
    assert bench.traffic_per_step("fp32", "mixed8000_rl14") is None    # another workload
    summ["kernel_hash"] = "0" * 16                                       # sources changed since
    f.write_text(json.dumps(summ))
    assert bench.traffic_per_step("fp32", wl) is None


"""Host-side pieces of bench.py: the multi-GPU refusal and the reduction of rocprofv3 PMC runs to the
traffic summary (synthetic counter files, no GPU)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

FIELDS = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=FIELDS)
        w.writeheader()
        for i, (disp, name, counter, value) in enumerate(rows):
            w.writerow({"Correlation_Id": i, "Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": value})


def test_write_traffic_scales_by_the_copy(tmp_path):
    gib_kib = (1 << 30) // 1024
    rows_k = "void moff::k_rows<256, 2, 0, false>(moff::RowArgs)"
    cols_k = "void moff::k_cols<256, 2, 8, 0, 0>(moff::ColArgs)"
    gemm_k = "void moff::k_rowgemm<256, 4>(moff::RgArgs)"
    rmf_k, cmf_k = "void moff::k_rows_mfma<0>(moff::RowArgs)", "void moff::k_cols_mfma<0, 0>(moff::ColArgs)"
    # counters are reported per instance: two instances of dispatch 7 sum to one dispatch's value
    _write(tmp_path / "pmc_fp32_FETCH_SIZE", [(7, rows_k, "FETCH_SIZE", 100), (7, rows_k, "FETCH_SIZE", 100),
                                              (9, rows_k, "FETCH_SIZE", 400), (8, cols_k, "FETCH_SIZE", 1000),
                                              (3, "other", "FETCH_SIZE", 5)])
    _write(tmp_path / "pmc_fp32_WRITE_SIZE", [(7, rows_k, "WRITE_SIZE", 3000), (8, cols_k, "WRITE_SIZE", 10)])
    _write(tmp_path / "pmc_gemm_fp16_FETCH_SIZE", [(4, gemm_k, "FETCH_SIZE", 50), (5, cols_k, "FETCH_SIZE", 900)])
    _write(tmp_path / "pmc_gemm_fp16_WRITE_SIZE", [(4, gemm_k, "WRITE_SIZE", 2000), (5, cols_k, "WRITE_SIZE", 20)])
    _write(tmp_path / "pmc_split_fp16_FETCH_SIZE", [(4, rmf_k, "FETCH_SIZE", 60), (5, cmf_k, "FETCH_SIZE", 800)])
    _write(tmp_path / "pmc_split_fp16_WRITE_SIZE", [(4, rmf_k, "WRITE_SIZE", 2500), (5, cmf_k, "WRITE_SIZE", 30)])
    # the copy reads half its bytes on FETCH_SIZE (scale 2) and all of them on WRITE_SIZE (scale 1)
    _write(tmp_path / "pmccopy_FETCH_SIZE", [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", gib_kib // 2)])
    _write(tmp_path / "pmccopy_WRITE_SIZE", [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", gib_kib)])
    out = tmp_path / "traffic.json"
    d = bench.write_traffic(str(tmp_path), launch_cs=4096, out_path=str(out))
    assert json.load(open(out)) == d
    assert d["src_hash"] == bench._src_hash()
    r, c = d["forms"]["fp32"]["k_rows"], d["forms"]["fp32"]["k_cols"]
    assert r["fetch_kib"] == 300 and r["write_kib"] == 3000           # (200 + 400) / 2 dispatches
    assert r["bytes_per_launch"] == (300 * 2 + 3000) * 1024
    assert c["bytes_per_launch"] == (1000 * 2 + 10) * 1024
    assert r["channel_samples_per_launch"] == 4096
    assert d["forms"]["gemm_fp16"]["k_rowgemm"]["bytes_per_launch"] == (50 * 2 + 2000) * 1024
    assert d["forms"]["gemm_fp16"]["k_cols"]["bytes_per_launch"] == (900 * 2 + 20) * 1024
    assert d["forms"]["split_fp16"]["k_cols_mfma"]["bytes_per_launch"] == (800 * 2 + 30) * 1024
    assert len(d["commands"]) == 2 * len(bench.TRAFFIC_FORMS) + 2


def test_traffic_needs_matching_sources(tmp_path, monkeypatch):
    d = {"src_hash": "not-this-build", "forms": {"fp32": {"k_rows": {"channel_samples_per_launch": 4096,
                                                                      "bytes_per_launch": 1}}}}
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "traffic.json").write_text(json.dumps(d))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "_src_hash", lambda: "this-build")
    assert bench._traffic("fp32", "k_rows", 4096) is None
    d["src_hash"] = "this-build"
    (prof / "traffic.json").write_text(json.dumps(d))
    assert bench._traffic("fp32", "k_rows", 4096) == 1
    assert bench._traffic("fp32", "k_rows", 2048) is None
    assert bench._traffic("gemm_fp16", "k_rows", 4096) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr

"""Host logic of bench.py (no GPU): the per-stage kernel table and roofline
bound, the selection of kernel instances in rocprofv3 counter files, and the
traffic record with its source-hash check."""
import csv
import json
import os

import pytest

import bench


def test_stage_table_and_roofline_bound():
    k = bench.stage_kernels(100)
    assert set(k) == {"jacvec", "correct", "div", "transform"}
    n3, np3 = 100 ** 3, 102 ** 3
    assert k["transform"][2] == 16.0 * n3 and k["div"][2] == 32.0 * n3
    assert k["jacvec"][2] == 96 * np3 and k["correct"][2] == 32 * n3 + 24 * np3
    f1, b1 = bench.transform_work(100)
    assert f1 == 2.0 * (50 * 50 + 50 * 50) * 100 * 100 and b1 == 16.0 * n3
    assert bench.stage_kernels(100, planes=True)["transform"][3] == 2 * f1
    # 6 flop/B is under the FP64 ridge (78.6 TF/s / 8 TB/s = 9.8): HBM-bound
    r = bench.roof_of(b1, f1, 12e-6)
    assert r["bound"] == "hbm" and r["achieved"] == pytest.approx(b1 / 12e-6 / 1e9)
    r = bench.roof_of(16.0 * 256 ** 3, bench.transform_work(256)[0], 100e-6)
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s"


def test_divergence_instances_are_told_apart():
    div = "void fvk::(anonymous namespace)::k_axis_sym<double, double, double, true, false, true, 4, 1, 1>(x)"
    plain = "void fvk::(anonymous namespace)::k_axis_sym<double, double, double, true, false, false, 4, 1, 0>(x)"
    assert bench._matches(div, "k_axis_sym:div") and not bench._matches(plain, "k_axis_sym:div")
    assert bench._matches(plain, "k_axis_sym") and not bench._matches(div, "k_axis_sym")
    assert bench._matches("k_jac_tiled<false, 4>(g)", "k_jac_tiled")


def _counters(folder, counter, rows):
    os.makedirs(folder)
    with open(os.path.join(folder, "b_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_ingest_scales_by_the_copy_and_checks_the_source_hash(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_JSON", str(tmp_path / "traffic.json"))
    names = {"k_jac_tiled": "k_jac_tiled<false, 4>(g)",
             "k_correct<": "k_correct<false, false>(g)",
             "div": "k_axis_sym<double, double, double, true, false, true, 4, 1, 1>(v)",
             "plain": "k_axis_sym<double, double, double, false, false, true, 4, 1, 0>(v)"}
    copy_kib = bench.COPY_BYTES / 1024.0
    # FETCH_SIZE counts half the bytes read (as measured on the box), WRITE_SIZE all
    _counters(str(tmp_path / "f"), "FETCH_SIZE", [(names[k], 1000.0) for k in names])
    _counters(str(tmp_path / "w"), "WRITE_SIZE", [(names[k], 500.0) for k in names])
    _counters(str(tmp_path / "cf"), "FETCH_SIZE", [("copy", copy_kib / 2), ("fill", 4.0)])
    _counters(str(tmp_path / "cw"), "WRITE_SIZE", [("copy", copy_kib), ("fill", 4.0)])
    bench.ingest_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                     str(tmp_path / "cw"), 100)
    rec = json.load(open(tmp_path / "traffic.json"))
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    expect = (1000.0 * 2 + 500.0) * 1024
    assert rec["kernels"]["k_axis_sym"]["traffic_bytes_per_launch"] == pytest.approx(expect)
    assert bench.traffic_entry(100, "transform") == pytest.approx(expect)
    assert bench.traffic_entry(256, "transform") is None            # another grid
    rec["kernels"]["k_axis_sym"]["source_sha256"] = "0" * 64          # an edited source
    json.dump(rec, open(tmp_path / "traffic.json", "w"))
    assert bench.traffic_entry(100, "transform") is None
    assert bench.traffic_entry(100, "jacvec") == pytest.approx(expect)

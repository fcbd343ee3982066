"""The profiler summaries' host logic (no GPU): tile shapes named from
kernel template names, HBM bytes per launch from FETCH_SIZE / WRITE_SIZE
dispatch rows scaled by the calibration copy, one traffic record per
workload with the other tile shapes merged into it, and the bench's lookup
of the record of the shape a line ran."""
import csv
import json
import os

import pytest

import bench
from paper_2209_08241_amd import profiling

HDR = ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value",
       "Start_Timestamp", "End_Timestamp"]


def _write_counters(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(HDR)
        for i, (kernel, grid, value) in enumerate(rows):
            w.writerow([i, kernel, grid, counter, value, 0, 1000])


@pytest.mark.parametrize("kernel,shape", [
    ("k_vec4<2, 1, 0>", "vec4"), ("k_vec4<3, 2, 18>", "vec4x2"), ("k_vec4<1, 4, 2>", "vec4x4"),
    ("k_vec4p<2, 1>", "vec4p2"), ("k_vec4w<2, 0, 128>", "vec4w128"),
    ("k_vec4w<2, 1, 64>", "vec4w64"), ("k_scalar<5, 0>", "scalar"), ("k_batch<2, 0>", None),
    ("k_vjp4_stack<2, 4, 8>", None), ("k_stack<2, 0>", None)])
def test_tile_shape_of_kernel(kernel, shape):
    assert profiling.tile_shape_of_kernel(kernel) == shape


def test_traffic_records_and_lookup(tmp_path, monkeypatch):
    calib = 1 << 30
    fetch, write = str(tmp_path / "f"), str(tmp_path / "w")
    # the calibration copy of 1 GiB reads cf FETCH_SIZE units and writes cw
    # WRITE_SIZE units (its four largest dispatches; a small one is ignored)
    cf, cw = 524288.0, 1048576.0
    fu, wu = calib / cf, calib / cw
    px = 1000
    rows_f = [("__amd_rocclr_copyBuffer", 1, cf)] * 4 + [("__amd_rocclr_copyBuffer", 1, 10.0)]
    rows_w = [("__amd_rocclr_copyBuffer", 1, cw)] * 4
    # two grid sizes of one kernel (two frame sizes) and a second tile shape
    rows_f += [("void bn::k_vec4<2, 1, 0>(bn::FrameArgs)", 250, 4.5 * px / fu)] * 3
    rows_w += [("void bn::k_vec4<2, 1, 0>(bn::FrameArgs)", 250, 13.0 * px / wu)] * 3
    rows_f += [("void bn::k_vec4<2, 1, 0>(bn::FrameArgs)", 999, 1e9)]
    rows_w += [("void bn::k_vec4<2, 1, 0>(bn::FrameArgs)", 999, 1e9)]
    rows_f += [("void bn::k_vec4p<2, 0>(bn::FrameArgs)", 125, 4.25 * px / fu)] * 2
    rows_w += [("void bn::k_vec4p<2, 0>(bn::FrameArgs)", 125, 13.0 * px / wu)] * 2
    _write_counters(fetch, "FETCH_SIZE", rows_f)
    _write_counters(write, "WRITE_SIZE", rows_w)
    out = str(tmp_path / "traffic_plainX.json")
    rec = profiling.traffic(fetch, write, "k_vec4<2, 1, 0>", px, "plainX", out, calib,
                            "copyBuffer", grid=250)
    assert rec["variant"] == "vec4" and rec["dispatches"] == {"fetch": 3, "write": 3}
    assert rec["hbm_bytes_per_launch"] == pytest.approx(17.5 * px)
    assert rec["read_bytes_per_pixel"] == pytest.approx(4.5)
    profiling.traffic(fetch, write, "k_vec4p<2, 0>", px, "plainX", out, calib, "copyBuffer",
                      grid=125)
    merged = json.load(open(out))
    assert merged["variant"] == "vec4"
    assert merged["other_tile_shapes"]["vec4p2"]["hbm_bytes_per_launch"] == \
        pytest.approx(17.25 * px)
    # the bench finds each shape's record while the sources hash the same
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    os.makedirs(tmp_path / "profiles")
    os.replace(out, tmp_path / "profiles" / "traffic_plainX.json")
    monkeypatch.setattr(bench, "kernel_hash", lambda sources=None: merged["kernel_hash"])
    assert bench.load_traffic("plainX", px, variant="vec4") == pytest.approx(17.5 * px)
    assert bench.load_traffic("plainX", px, variant="vec4p2") == pytest.approx(17.25 * px)
    assert bench.load_traffic("plainX", px, variant="vec4w64") is None
    monkeypatch.setattr(bench, "kernel_hash", lambda sources=None: "other")
    assert bench.load_traffic("plainX", px, variant="vec4") is None

"""Host-side checks of the measurement arithmetic: the method's per px·label
work behind the bench line's roofline, and the conversion of rocprofv3 byte
counters into HBM bytes per launch (no GPU needed)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1803_00005_amd import profile_summary, synth  # noqa: E402


def test_method_model_of_the_named_workloads():
    """Cost in and Z out per px·label plus the guidance read and label write
    spread over the labels; flops of the product M c, the two box filters,
    the covariances and output, plus the per-pixel statistics and inverse."""
    c2 = bench.method_model(synth.WORKLOADS["voronoi450x375_n9_L60"])
    assert c2["bytes"] == pytest.approx(4 + 4 + 16 / 60)
    assert c2["flops"] == pytest.approx(2 * 81 + 80 + 63 + (729 + 4 * 9 * 12 / 2) / 60)
    assert round(c2["flops"]) == 321
    c3 = bench.method_model(synth.WORKLOADS["voronoi1242x375_n19_L128"])
    assert c3["bytes"] == pytest.approx(8.125)
    assert round(c3["flops"]) == 1075
    bf = bench.method_model(synth.WORKLOADS["voronoi1242x375_n19_L128_bf16"])
    assert bf["bytes"] == pytest.approx(6.125)      # 16-bit cost reads
    assert bf["flops"] == pytest.approx(c3["flops"])


def test_roofline_fractions():
    """frac is the algorithmic bytes of one launch over its time against
    8 TB/s; the method's intensity lies above the ridge, so the binding roof
    is the vector ALU."""
    w = synth.WORKLOADS["voronoi450x375_n9_L60"]
    units, ms = float(w.pixel_labels), 0.2854
    r = bench.method_roofline(w, "out_kernel", units, ms, None, None, 0.548)
    mm = bench.method_model(w)
    assert r["achieved"] == pytest.approx(units * mm["bytes"] / (ms * 1e-3) / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["frac"] == pytest.approx(0.0367, abs=5e-4)
    assert r["alu"]["frac"] == pytest.approx(units * mm["flops"] / (ms * 1e-3) / 157.3e12)
    assert r["binding_roof"] == "alu"
    assert r["traffic"] is None


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "1_counter_collection.csv"), "w", newline="") as fh:
        wr = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        wr.writeheader()
        for k, c, v in rows:
            wr.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_counter_calibration(tmp_path):
    """Raw FETCH_SIZE / WRITE_SIZE (KiB per dispatch) are scaled by what the
    same counters read for a 1 GiB sum and a 1 GiB fill."""
    out_k = "void hgf::out_kernel<9, 1, 9, 64, 8, true>(float const*, float const*)"
    sum_k = "void at::native::reduce_kernel<512, 1, at::native::ReduceOp<float, sum_functor>>"
    fill_k = "void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>>"
    fdir, wdir = str(tmp_path / "fetch"), str(tmp_path / "write")
    # the sum's fetch counter reads half the bytes it moved, the fill's write all
    _write_counters(fdir, [(sum_k, "FETCH_SIZE", 2 ** 19), (out_k, "FETCH_SIZE", 1000.0),
                           (out_k, "FETCH_SIZE", 1200.0)])
    _write_counters(wdir, [(fill_k, "WRITE_SIZE", 2 ** 20), (out_k, "WRITE_SIZE", 100.0),
                           (out_k, "WRITE_SIZE", 100.0)])
    out = str(tmp_path / "c.json")
    profile_summary.counters(fdir, wdir, out, "w", "cmd")
    rec = json.load(open(out))
    assert rec["fetch_factor"] == pytest.approx(2.0)
    assert rec["write_factor"] == pytest.approx(1.0)
    k = rec["kernels"]["out_kernel"]
    assert k["dispatches"] == 2
    assert k["hbm_bytes_per_launch"] == pytest.approx(1024 * (1100.0 * 2.0 + 100.0))
    assert k["source_hash"] == profile_summary.source_hash("out_kernel")
    assert "calibration_sum" not in rec["kernels_full"]

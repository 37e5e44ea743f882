"""Every bench.py workload at a tiny size: the JSON line keeps its contract
(metric, value, unit, roofline where the workload reports one) and is
serialisable.  Throughput values are not checked, only that they are
positive and finite."""
import argparse
import json
import math

import pytest

import bench

pytestmark = pytest.mark.gpu


def _args(workload, frames, **kw):
    a = dict(gpus=1, steps=2, warmup=1, workload=workload, r=8, backend="auto", frames=frames,
             no_cpu_baseline=True, no_variants=False, cpu_frames=1, calibrate_copy=False, q=None, qp=None,
             no_c2=True, no_graphs=False)
    a.update(kw)
    return argparse.Namespace(**a)


def _run(workload, frames, **kw):
    import torch

    import paper_1606_05562_amd as A
    fn = {"target": bench.bench_target, "luma": bench.bench_luma, "ragged": bench.bench_ragged,
          "residual": bench.bench_residual, "rd": bench.bench_rd, "sweep": bench.bench_sweep,
          "vector": bench.bench_vector}[workload]
    res = fn(_args(workload, frames, **kw), A, torch)
    line = json.loads(json.dumps(res))  # plain JSON types only
    for key in ("metric", "value", "unit", "n_gpus", "config", "higher_is_better"):
        assert key in line, key
    assert line["n_gpus"] == 1
    return line


def _positive(v):
    return isinstance(v, (int, float)) and math.isfinite(v) and v > 0


def _check_frames_line(line, steps=2):
    assert _positive(line["value"])
    r = line["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel_ms_mean", "kernel_ms_median"):
        assert key in r, key
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    # the persistent kernel of every timed step, and no longer than the step
    assert r["kernel_launches"] == steps
    assert 0 < r["kernel_ms_mean"] <= line["ms_per_step"] * 1.001
    assert line["parity"]["ok"] is True
    assert isinstance(line["config"]["seed"], int) and "form" in line["config"]


def test_bench_luma_small():
    line = _run("luma", 2, no_cpu_baseline=False)
    _check_frames_line(line)
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and _positive(cb["value"]) and cb["cores"] >= 1
    assert _positive(cb["single_thread"]["value"]) and cb["single_thread"]["cores"] == 1
    assert cb["cpu_model"] and cb["host_nproc"] >= 1
    assert all(_positive(v) for v in line["variants"].values())


def test_bench_target_small():
    line = _run("target", 1)
    _check_frames_line(line)
    assert line["config"]["width"] == 3840 and line["config"]["height"] == 2160
    assert all(_positive(v) for v in line["variants"].values())


def test_bench_ragged_small():
    line = _run("ragged", 4)
    assert _positive(line["value"]) and line["roofline"]["bound"] == "hbm"
    lay = line["config"]["layouts"]
    assert set(lay) == {"lines128", "packed16"}
    assert lay["lines128"]["plan"]["rows_line_aligned"] is True
    assert all(_positive(x["gpix_s"]) and x["parity"]["ok"] is True for x in lay.values())
    assert lay["packed16"]["bytes"] <= lay["lines128"]["bytes"]


def test_bench_residual_small():
    line = _run("residual", 1)
    per_q = line["config"]["per_q"]
    for q in (8, 16, 32):
        for form in ("auto", "mfma", "valu"):
            assert _positive(per_q[f"q{q}_{form}_graphs_gsample_s"])
            assert _positive(per_q[f"q{q}_{form}_calls_gsample_s"])
            assert _positive(per_q[f"q{q}_{form}_one_launch_gsample_s"])
        assert per_q[f"q{q}_mfma_plan"]["levels_backend"] == "mfma"
        assert per_q[f"q{q}_valu_plan"]["levels_backend"] == "valu"
        assert per_q[f"q{q}_auto_plan"]["levels_backend"] in ("mfma", "valu")
    # the headline is the autotuned plan's, and names the arithmetic it ran
    assert line["value"] == per_q["q16_auto_calls_gsample_s"] and "one call per frame" in line["metric"]
    assert ("MFMA" in line["dtype"]) == (per_q["q16_auto_plan"]["levels_backend"] == "mfma")
    r = line["roofline"]
    assert r["bound"] == "hbm" and _positive(r["achieved"]) and abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    assert r["kernel"].startswith("k_mfma_resid") and r["kernel_launches"] == line["steps"]
    assert line["parity"]["ok"] is True
    # counters are committed for the full 120-frame stream only
    assert r["traffic"] is None and r["compute"] is None


def test_bench_residual_one_launch_only():
    """--no-graphs: the one-launch calls alone, parity from the one launch."""
    line = _run("residual", 1, q=16, no_graphs=True)
    per_q = line["config"]["per_q"]
    assert "q16_mfma_graphs_gsample_s" not in per_q and "one launch" in line["metric"]
    assert line["value"] == per_q["q16_auto_one_launch_gsample_s"]
    assert line["parity"]["ok"] is True and line["roofline"]["kernel"].startswith("k_mfma_resid")


def test_bench_residual_one_step_with_copy_calibration():
    line = _run("residual", 1, q=8, calibrate_copy=True)
    per_q = line["config"]["per_q"]
    assert _positive(per_q["q8_mfma_graphs_gsample_s"]) and "q16_mfma_graphs_gsample_s" not in per_q
    assert line["value"] == per_q["q8_auto_calls_gsample_s"]
    r = line["roofline"]
    assert "q = 8" in r["timing"] and r["calibration_copy_bytes"] > 0


def test_bench_rd_one_point_with_copy_calibration():
    line = _run("rd", 1, qp=32, calibrate_copy=True)
    pts = line["config"]["rd_curve"]
    assert [p["qp"] for p in pts] == [32] and line["value"] == pts[0]["mfma_gsample_s"]
    r = line["roofline"]
    assert "QP 32" in r["timing"] and r["calibration_copy_bytes"] > 0


def test_bench_rd_small():
    line = _run("rd", 1)
    pts = line["config"]["rd_curve"]
    assert [p["qp"] for p in pts] == [22, 27, 32, 37]
    assert line["value"] == pts[1]["mfma_gsample_s"]
    assert all(p["mfma_plan"]["levels_backend"] == "mfma" and _positive(p["valu_gsample_s"]) for p in pts)
    # the committed counters were taken on 8 frames: none reported for 1
    assert line["roofline"]["traffic"] is None and line["roofline"]["compute"] is None
    # coarser steps never cost more bits
    bits = [p["bits_per_sample"] for p in pts]
    assert all(a >= b for a, b in zip(bits, bits[1:]))
    assert line["roofline"]["bound"] == "hbm" and _positive(line["roofline"]["achieved"])


def test_bench_sweep_small():
    line = _run("sweep", 2)
    rows = line["config"]["rows"]
    assert rows[0]["r"] == 1 and rows[-1]["r"] == 255
    # retaining more coefficients never lowers the mean PSNR of either transform
    pa = [r["psnr_approx_db"] for r in rows if r["psnr_approx_db"] is not None]
    assert all(a <= b + 1e-9 for a, b in zip(pa, pa[1:]))


def test_bench_vector_small():
    line = _run("vector", 1)
    assert _positive(line["value"]) and line["roofline"]["bound"] == "hbm"
    assert set(line["config"]["per_direction"]) == {"forward", "inverse"}

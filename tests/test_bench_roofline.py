"""The roofline object of the benchmark line (host arithmetic, no GPU):
achieved and frac come from the algorithmic work of the step, the bound is
the roof with the larger algorithmic fraction, and measured traffic is only
reported beside them."""
import pytest

import bench


def test_step_roofline_from_algorithmic_work():
    # 4He relativistic, step 3: 3.29e8 complex FMAs per lane, stage 2 read and
    # stage 3 written once in float, 768 lanes, 64 ms, 455 GB measured
    flops = 329119200 * 8.0 * 768
    r = bench.step_roofline(flops, 6586560, 1828440, 8, 792 * 32, 768, 64.0, traffic=455e9)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["peak"] == bench.VALU_PEAK_TFLOPS
    assert r["achieved"] == pytest.approx(flops / 0.064 / 1e12, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.VALU_PEAK_TFLOPS, rel=1e-3)
    alg = ((6586560 + 1828440) * 8 + 792 * 32) * 768
    assert r["algorithmic_bytes_per_launch"] == alg
    assert r["hbm_frac_algorithmic"] == pytest.approx(alg / 0.064 / 1e9 / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["hbm_frac_algorithmic"] < r["frac"]
    # the measured traffic: beside the algorithmic figures, never in them
    assert r["traffic"] == 455e9
    assert r["measured_traffic_gbps"] == pytest.approx(455e9 / 0.064 / 1e9, rel=1e-3)
    assert r["traffic_over_algorithmic"] == pytest.approx(455e9 / alg, rel=1e-2)


def test_step_roofline_bound_by_bytes():
    # little arithmetic per byte: the HBM roof binds, achieved is algorithmic GB/s
    r = bench.step_roofline(1e9, 10**9, 10**9, 16, 0, 64, 10.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
    alg = 2 * 10**9 * 16 * 64
    assert r["achieved"] == pytest.approx(alg / 0.010 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["traffic"] is None and "measured_traffic_gbps" not in r

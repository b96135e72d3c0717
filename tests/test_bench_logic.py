"""Host logic of bench.py: which kernel the roofline object describes, and which traffic
record goes with it (no GPU: synthetic timing dictionaries)."""
from __future__ import annotations

import os
import sys
import types

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _w(n, d, precision):
    return types.SimpleNamespace(d=d, precision=precision, graph=types.SimpleNamespace(n=n), name="x")


def _k(ms_per_launch, launches=3):
    return {"launches": launches, "ms_total": ms_per_launch * launches, "ms_per_launch": ms_per_launch}


N1M = 1_000_000 * 999_999 // 2


def test_bf16_full_sweep_taken_when_it_ran_and_dominates():
    r = {"N": N1M, "kernels": {"gram_screen": _k(42.7), "full_sweep": _k(741.0)}}
    roof = bench.roofline_of(_w(1_000_000, 16, "bf16"), r, 3)
    assert roof["kernel"].startswith("k_sweep_mfma16<true>")
    assert roof["flops_per_pair"] == bench.flops_per_pair(16) == 7 * 16 + 31
    assert roof["peak"] == bench.PEAK_FP32_TFLOPS
    assert roof["frac"] == pytest.approx(143 * N1M / 0.741 / 1e12 / 157.3)


def test_bf16_gated_exit_is_not_taken_for_the_full_sweep():
    # a launch that returned at once: far shorter than every pair needs at the FP32 peak,
    # even when the screen is shorter still
    r = {"N": 5_000 * 4_999 // 2, "kernels": {"gram_screen": _k(0.004), "full_sweep": _k(0.009)}}
    roof = bench.roofline_of(_w(5_000, 128, "bf16"), r, 3)
    assert roof["kernel"].startswith("k_gram_screen")
    assert roof["flops_per_pair"] == 2 * 128 and roof["peak"] == bench.PEAK_BF16_TFLOPS


def test_bf16_screen_taken_when_it_dominates():
    n = 100_000
    r = {"N": n * (n - 1) // 2, "kernels": {"gram_screen": _k(1.0), "full_sweep": _k(0.0124)}}
    roof = bench.roofline_of(_w(n, 128, "bf16"), r, 3)
    assert roof["kernel"].startswith("k_gram_screen")


def test_fp32_kernel_names():
    n = 1_000_000
    r = {"N": N1M, "kernels": {"sweep": _k(740.0)}}
    assert bench.roofline_of(_w(n, 16, "fp32"), r, 3)["kernel"].startswith("k_sweep_mfma16<false>")
    assert bench.roofline_of(_w(100_000, 128, "fp32"), {"N": 1, "kernels": {"sweep": _k(47.0)}}, 3)[
        "kernel"].startswith("k_sweep_mfma_wide<128, false>")


def test_traffic_keys():
    assert bench.traffic_kernel_of(_w(3_400, 2, "fp32")) == "gempe::k_iter<2>"
    assert bench.traffic_kernel_of(_w(1_000_000, 16, "fp32")) == "gempe::k_sweep_mfma16<false>"
    assert bench.traffic_kernel_of(_w(100_000, 128, "fp32")) == "gempe::k_sweep_mfma_wide<128, false>"
    k = bench.traffic_kernel_of(_w(100_000, 128, "bf16"))
    assert k.startswith("_ZN5gempe13k_gram_screenILi128ELi8E")
    assert bench.sources_of(k) == bench.SCREEN_SOURCES
    assert bench.sources_of("gempe::k_iter<2>") == bench.TRAFFIC_SOURCES


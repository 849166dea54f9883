"""The benchmark's host-side contract, checked without a GPU: more than one GPU is refused with a message, and
the roofline entries compute achieved = units x per-unit work / duration against MI355X's published peaks."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_peaks_are_the_published_ones():
    assert bench.HBM_PEAK_GBPS == pytest.approx(8000.0)
    assert bench.BF16_PEAK_TFLOPS == pytest.approx(2500.0)
    assert bench.FP32_VECTOR_PEAK_TFLOPS == pytest.approx(157.3)


def test_box_and_pairs_rooflines():
    # 1e9 sphere tests of 10 flop in 1 ms: 10 TFLOP/s
    r = bench.box_roofline(1e9, 1.0)
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s" and r["kernel"] == "k_box"
    assert r["achieved"] == pytest.approx(10.0)
    assert r["frac"] == pytest.approx(10.0 / 157.3)
    assert r["units"] == 10**9 and r["time_ms"] == 1.0
    # 1e6 pairs of 768 flop in 0.5 ms: 1.536 TFLOP/s
    p = bench.pairs_roofline(1e6, 0.5)
    assert p["achieved"] == pytest.approx(1.536)
    assert p["frac"] == pytest.approx(1.536 / 157.3)
    assert bench.box_roofline(5, 0.0)["achieved"] is None


def test_finish_roofline_counts_algorithmic_bytes():
    # 100 B per query + 36 B per pair + the span coefficients
    r = bench.finish_roofline(1000, 2500, 48_000, 0.001)
    assert r["algorithmic_bytes"] == 100 * 1000 + 36 * 2500 + 48_000
    assert r["achieved"] == pytest.approx(r["algorithmic_bytes"] / 1e-6 / 1e9)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["frac"] == pytest.approx(r["achieved"] / 8000.0)


def test_screen_roofline_method_and_padded_work():
    r = bench.screen_roofline(1e12, 100.0, 200.0)
    assert r["achieved"] == pytest.approx(1e12 * 38 / 0.1 / 1e12)
    assert r["frac_padded_k"] == pytest.approx(1e12 * 64 / 0.1 / 1e12 / 2500.0)
    assert r["frac_whole_call"] == pytest.approx(r["frac"] / 2.0)

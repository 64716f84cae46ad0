"""Host logic of bench.py (no GPU): the single-GPU refusal, the per-pair
operation counts and peaks behind `roofline`, and the committed rocprofv3
summaries it reads (keyed by the hash of the launch-shaping sources)."""
import os
import re
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C4 = "d3_N30000_chi0.45_w"
C4_PAIRS = 40494 * 30000  # M x N of d=3, N=30000, chi=0.45


def test_more_than_one_gpu_is_refused_before_any_device_work():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr and r.stdout == ""


def test_per_pair_counts_and_peaks():
    # n~ pass: b z^t and b conj(z^t) share four lazy dd products (4 mul, 12 fma per
    # two wavevectors) and four TwoSums with their error terms (32 add), plus two
    # lazy accumulations (8 add each) per wavevector
    assert bench.OPS_PER_PAIR_MIX["nk"] == (16 + 16, 4 // 2, 12 // 2)
    # gradient pass: a lazy complex product (2 x (8 add, 2 mul, 6 fma)), the lazy
    # dot product v (S c - C s) (8, 2, 6) and two lazy accumulations (8 add each)
    assert bench.OPS_PER_PAIR_MIX["grad"] == (16 + 8 + 16, 4 + 2, 12 + 6)
    assert bench.OPS_PER_PAIR == {"nk": 40, "grad": 64}
    assert bench.FLOPS_PER_PAIR == {"nk": 46, "grad": 82}
    assert bench.PEAK_FP64_OPS == pytest.approx(39.3216e12)
    assert bench.PEAK_FP64_FLOPS == pytest.approx(78.6432e12)


def stats_avg_us(name: str, kernel_prefix: str) -> float:
    with open(os.path.join(ROOT, "profiles", name)) as fh:
        for line in fh:
            if line.startswith(f"| void ss::{kernel_prefix}"):
                return float(line.split("|")[3])
    raise AssertionError(f"{kernel_prefix} not in {name}")


def test_roofline_from_launch_times():
    avg_ms = stats_avg_us(f"kernel_stats_{C4}.md", "k_grad<3>") / 1e3
    r = bench.roofline("grad", "k_grad", 10, 10 * avg_ms, 10 * C4_PAIRS, C4)
    assert r["avg_launch_ms"] == pytest.approx(avg_ms)
    assert r["achieved"] == pytest.approx(82 * C4_PAIRS / (avg_ms * 1e-3) / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6432)
    assert r["issue"]["frac"] == pytest.approx(64 * C4_PAIRS / (avg_ms * 1e-3) / 39.3216e12)
    # the committed summaries are of the current sources: traffic and executed flops
    # are read, and the executed count covers at least the inner loop's
    assert r["traffic"] is not None and r["executed"] is not None
    assert r["executed"]["flops_per_launch"] >= 82 * C4_PAIRS
    # a roofline fraction is a fraction
    assert 0.0 < r["frac"] < r["issue"]["frac"] < 1.0


def test_profiles_are_of_the_current_sources():
    h = bench.kernel_source_hash()
    for name in sorted(os.listdir(os.path.join(ROOT, "profiles"))):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            text = fh.read()
        m = re.search(r"kernel_source_hash: ([0-9a-f]{16})", text)
        assert m and m.group(1) == h, name


def test_summaries_ignored_for_other_sources(monkeypatch):
    assert bench.read_traffic("k_nk", C4) is not None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.read_traffic("k_nk", C4) is None
    assert bench.read_fp64_flops("k_grad", C4) is None


def test_counter_calibration_is_sane():
    # on a 1 GiB device copy FETCH_SIZE reads half of the copied bytes (scale ~2)
    # and WRITE_SIZE all of them (scale ~1); per-launch bytes are the scaled sum
    # (of the rounded figures the summary prints)
    for kernel in ("k_nk", "k_grad"):
        rec = bench.read_profile(f"{kernel}_{C4}_counters.txt")
        fs, ws = float(rec["fetch_scale"]), float(rec["write_scale"])
        assert 1.5 < fs < 2.5 and 0.9 < ws < 1.1
        total = (float(rec["fetch_kib_per_dispatch"]) * fs + float(rec["write_kib_per_dispatch"]) * ws) * 1024
        assert float(rec["hbm_bytes_per_launch"]) == pytest.approx(total, rel=1e-4)

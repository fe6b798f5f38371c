"""Host logic of bench.py (no GPU): the algorithmic work per element, the
roofline object, the counter-bytes guard and the one-GPU refusal."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_split_work_2d_p4():
    # n_p = 22, n_f = 5, n_c = 4: 4 * 2 * 4 * 22^2 + 500 * 22 flops;
    # 4 * 22 * (8 + 8) + 12 * 8 + 3 * 5 * 4 + 4 bytes
    fl, by = bench.work_split(2, 22, 5)
    assert fl == 15488 + 11000
    assert by == 1408 + 96 + 60 + 4
    fl32, by32 = bench.work_split(2, 22, 5, out_bytes=4)
    assert fl32 == fl and by32 == by - 4 * 22 * 4


def test_work_3d_families():
    fl, by = bench.work_split(3, 60, 12)
    assert fl == 4 * 3 * 5 * 3600 + 500 * 60
    assert by == 5 * 60 * 16 + 80 + 4 * 12 * 4 + 4
    assert bench.work_split(3, 60, 12, curved=True)[1] == by + 20 * 8
    fh, bh = bench.work_hadamard(3, 60, 12)
    assert fh == 175 * 60 * 59 / 2 + 2 * 3 * 5 * 3600 + 500 * 60 and bh == by
    fv, bv = bench.work_vjp(fl, 3, 60, 12)
    assert fv == 2 * fl and bv == 3 * 5 * 60 * 8 + 80 + 4 * 12 * 4 + 4
    fn, bn = bench.work_ns(60, 12)
    assert fn == fl + 4 * 3 * 5 * 3600 + 2 * 60 * 4 * 12 * 3 * 5 + 150 * 60 and bn == by


def test_roofline_bound_and_fraction():
    # compute-bound: the FP64 peak
    r = bench.roofline(26488.0, 1568, 32768, 56e-6, bench.PEAK_F64, "alu", "x", 0, "k")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(26488.0 * 32768 / 56e-6 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    # a low-intensity call is HBM-bound
    r = bench.roofline(100.0, 1000, 1000, 1e-6, bench.PEAK_F64, "alu", "x", 0, "k")
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(1000 * 1000 / 1e-6 / 1e9)


def test_counter_bytes_need_the_same_sources(monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC", {"tri_p4/fp64_split/v0": 1.0e6})
    monkeypatch.setattr(bench, "TRAFFIC_SHA", bench.kernel_source_hash())
    assert bench.measured_traffic("tri_p4/fp64_split", 0) == 1.0e6
    assert bench.measured_traffic("tri_p4/fp64_split", 1) is None
    monkeypatch.setattr(bench, "TRAFFIC_SHA", "0" * 16)
    assert bench.measured_traffic("tri_p4/fp64_split", 0) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr

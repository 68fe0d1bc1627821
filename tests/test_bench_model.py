"""CPU checks of the benchmark's work model: per-element flops (Table 2 for F_ax, Table 3 for
F_geo) and algorithmic bytes, and the time-based roofline (Sec. 3.4) built from them."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_flops_per_element_n7():
    f_ax, f_geo = bench.flops_per_element(7, "tri")
    assert f_ax == 12 * 8**4 + 15 * 8**3 == 56832
    assert f_geo == 72 * 8 + 45 * 64 + 80 * 512 == 44416
    assert bench.flops_per_element(7, "partial")[1] == 72 * 8 + 45 * 64 + 60 * 512
    assert bench.flops_per_element(7, "para")[1] == 7 * 512
    assert bench.flops_per_element(7, "stored")[1] == 0
    # columns share the geometry
    f3, g3 = bench.flops_per_element(7, "tri", nrhs=3)
    assert f3 == 3 * f_ax and g3 == f_geo


def test_bytes_per_element():
    assert bench.bytes_per_element(7, "tri") == 2 * 512 * 8 + 24 * 8 == 8384
    assert bench.bytes_per_element(7, "stored") == 2 * 512 * 8 + 6 * 512 * 8
    assert bench.bytes_per_element(7, "partial") == 8384 + 512 * 8
    assert bench.bytes_per_element(7, "helm") == 8384 + 2 * 512 * 8
    assert bench.bytes_per_element(3, "tri", fpsize=4) == 2 * 64 * 4 + 192
    assert bench.bytes_per_element(7, "tri", nrhs=3) == 6 * 512 * 8 + 192


def test_roofline():
    # stored factors: 64 B per DOF at 8 TB/s = 125 GDOF/s, HBM-bound
    r, bound = bench.roofline_gdofs(7, "stored")
    assert bound == "hbm" and r == pytest.approx(125.0)
    # on the fly at N = 7: compute-bound, (F_ax + F_geo) / 78.6 TF per element
    r, bound = bench.roofline_gdofs(7, "tri")
    assert bound == "alu" and r == pytest.approx(512 / (101248 / 78.6e12) / 1e9)
    # N = 3 on the fly: HBM-bound (19 B per DOF)
    r, bound = bench.roofline_gdofs(3, "tri")
    assert bound == "hbm" and r == pytest.approx(64 / (1216 / 8e12) / 1e9)

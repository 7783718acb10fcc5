"""The metric arithmetic against the paper's own Table 2 (Sec. 4.3 definitions:
B_node = 2 q s_d, P_B = B_node P_LUPS, U_B = P_B / B_peak, B_peak = 547.68 GB/s)."""
import json
import os

import pytest

from paper_2108_13241_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_table2.json")


def test_table2_rows():
    g = json.load(open(GOLDEN))
    peak = g["B_peak_GBps"]
    for row in g["rows"]:
        b = metrics.paper_bytes_per_node(row["s_d"], g["q"])
        assert b == 2 * 9 * row["s_d"]
        # printed GLUPS carry 2 decimals: P_B agrees within that rounding
        pb = metrics.bandwidth_gbps(row["glups"], b)
        assert abs(pb - row["gbps"]) <= 0.005 * b + 0.5
        ub = metrics.utilisation(row["gbps"], peak)
        assert abs(ub - row["U_B"]) <= 0.005 * b / peak + 5e-4


def test_table2_coefficients():
    """U_B = C P_GLUPS with C = 0.131 (FP32) and 0.263 (FP64) on the paper's GPU."""
    g = json.load(open(GOLDEN))
    for prec, s_d in (("fp32", 4), ("fp64", 8)):
        c = metrics.paper_bytes_per_node(s_d) / g["B_peak_GBps"]
        assert c == pytest.approx(g["C_coefficients"][prec], abs=6e-4)


def test_build_byte_counts():
    assert metrics.bytes_per_node("f64") == 145
    assert metrics.bytes_per_node("f32") == 73
    assert metrics.bytes_per_node("f16s") == 37
    assert metrics.bytes_per_node("f32", drag=True) == 77
    assert metrics.glups(4096 * 4096, 1000, 0.5) == pytest.approx(33.554432)

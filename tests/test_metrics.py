"""Byte and intensity accounting pinned to the paper's printed tables."""
import json
import os

from paper_2105_14156_amd import metrics

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_csr_bytes.json")))


def test_input_csr_table():
    # Table "data_sizes_input": row pointer, column index, data array, total.
    g = GOLD
    assert (g["rows"] + 1) * 4 == g["input_row_ptr_bytes"]
    assert g["nnz_a"] * 4 == g["input_col_idx_bytes"]
    assert g["nnz_a"] * g["value_bytes"] == g["input_data_bytes"]
    assert metrics.csr_bytes(g["rows"], g["nnz_a"], g["value_bytes"]) == g["input_total_bytes"]


def test_output_csr_table():
    # Table "data_sizes_output", with the paper's int32 row pointer.
    g = GOLD
    assert g["nnz_c"] * 4 == g["output_col_idx_bytes"]
    assert g["nnz_c"] * g["value_bytes"] == g["output_data_bytes"]
    assert metrics.csr_bytes(g["rows"], g["nnz_c"], g["value_bytes"]) == g["output_total_bytes"]


def test_algorithmic_bytes_is_paper_total_plus_int64_row_ptr():
    g = GOLD
    tot = metrics.algorithmic_bytes(g["rows"], g["rows"], g["nnz_a"], g["nnz_b"], g["nnz_c"], g["value_bytes"])
    paper = 2 * g["input_total_bytes"] + g["output_total_bytes"]
    assert tot == paper + (g["rows"] + 1) * 4   # C.row_ptr widened from int32 to int64


def test_arithmetic_intensity_matches_printed_value():
    g = GOLD
    products = g["cf"] * g["nnz_c"]          # cf = products / nnz(C)
    ai = metrics.arithmetic_intensity(products, g["nnz_a"], g["nnz_b"], g["nnz_c"], g["element_bytes"])
    assert round(ai, 2) == g["ai_printed"]
    assert abs(ai - 0.0933) < 1e-4
    # the 2 x products reading of "flop" would not round to the printed 0.09
    assert round(2 * ai, 2) != g["ai_printed"]
    assert metrics.arithmetic_intensity(products, g["nnz_a"], g["nnz_b"], g["nnz_c"], g["element_bytes"]) <= g["cf"] / g["element_bytes"]


def test_gflops():
    assert metrics.gflops(10**9, 1.0) == 2.0

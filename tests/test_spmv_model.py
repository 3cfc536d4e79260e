"""The paper's SpMV cache model (closed form) against the values it prints."""
import json
import os

import pytest

from oracle import spmv_model as M

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_predicted_speedups_match_printed_values():
    with open(os.path.join(GOLD, "paper_spmv_model.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        assert round(M.predicted_speedup(c["w"]), 2) == c["speedup_printed"]
    assert M.predicted_speedup(1e9) == pytest.approx(g["limit"], rel=1e-6)


@pytest.mark.parametrize("w", [1, 5, 7, 27])
def test_byte_ratio_is_the_speedup(w):
    n = 1000
    assert M.fp64_no_reuse_bytes(n, w) / M.fp32_perfect_cache_bytes(n, w) == pytest.approx(
        M.predicted_speedup(w))
    assert M.fp64_no_reuse_bytes(n, w) == 20 * w * n
    assert M.fp32_perfect_cache_bytes(n, w) == (8 * w + 4) * n


def test_algorithmic_spmv_bytes():
    # 1000x1000 5-point grid: 8 nnz + 4 (n+1) + 8 n bytes in fp32
    n, nnz = 1_000_000, 4_996_000
    assert M.spmv_bytes(n, nnz, 4) == 8 * nnz + 4 * (n + 1) + 8 * n
    assert M.spmv_bytes(n, nnz, 8) == 12 * nnz + 4 * (n + 1) + 16 * n

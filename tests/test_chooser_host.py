"""Host logic of the parameter chooser (no GPU): label encoding, snapping of
network outputs to the configuration grid, the per-iteration cost model that
turns a time budget into an iteration budget, and the sweep-record loader."""
import json
import math

import numpy as np

from paper_2109_01232_amd import chooser as C


def test_encode_snap_roundtrip_on_every_grid_point():
    for cfg in C.grid():
        assert C.snap(C.encode(*cfg)) == cfg


def test_snap_clamps_and_rounds_in_log_space():
    assert C.snap([100.0, 100.0, 100.0]) == (max(C.M_GRID), max(C.CAP_GRID), max(C.DEG_GRID))
    assert C.snap([-100.0, -100.0, -100.0]) == (min(C.M_GRID), min(C.CAP_GRID), min(C.DEG_GRID))
    # between 50 and 75 in log2 space: log2(61.2) is the midpoint
    assert C.snap([math.log2(60.0), 0.0, 0.0])[0] == 50
    assert C.snap([math.log2(63.0), 0.0, 0.0])[0] == 75


def test_default_is_on_the_grid():
    assert C.DEFAULT in C.grid()
    assert len(C.grid()) == len(C.M_GRID) * len(C.CAP_GRID) * len(C.DEG_GRID)


def test_iteration_cost_model_is_monotone():
    n, nnz = 10**6, 5 * 10**6
    base = C._iter_cost((50, 1, 0), n, nnz)
    assert C._iter_cost((100, 1, 0), n, nnz) > base
    assert C._iter_cost((50, 1, 10), n, nnz) > base
    # one polynomial degree costs one SpMV: 8 bytes per nonzero + 12 per row
    d = C._iter_cost((50, 1, 1), n, nnz) - base
    assert d == 8.0 * nnz + 12.0 * n


def test_load_records_filters_and_sorts(tmp_path):
    recs = [{"seed": 3, "best": [50, 1, 0]}, {"seed": 1, "best": None}, {"seed": 2, "best": [30, 2, 10]}]
    p = tmp_path / "sweep.jsonl"
    p.write_text("\n".join(json.dumps(r) for r in recs) + "\n")
    out = C.load_records([str(p)])
    assert [r["seed"] for r in out] == [2, 3]


def test_label_encoding_scale():
    y = np.array([C.encode(*cfg) for cfg in C.grid()])
    # targets stay O(1) so the tanh network needs no output scaling
    assert np.all(np.abs(y) <= 8.0)

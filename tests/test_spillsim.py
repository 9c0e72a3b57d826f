"""Pins for the spill-policy simulator (read-sort-write run generation with an
in-memory index of unique keys): a hand-worked case, closed forms, and the
paper's no-spill condition."""
import numpy as np
import pytest

import datagen
from oracle import spillsim


def test_hand_worked_case():
    # batches {1,2} {1,3} {4,5} {1,2}; capacity 3:
    #   {1,2} -> index {1,2}; {1,3} -> {1,2,3}; {4,5} -> spill 3, index {4,5};
    #   {1,2} -> union has 4 > 3 keys -> spill 2, index {1,2}
    keys = np.array([1, 2, 1, 3, 4, 5, 1, 2], np.uint64)
    r = spillsim.simulate(keys, batch_rows=2, capacity=3)
    assert r == {"runs": 2, "spilled_rows": 5, "run_sizes": [3, 2], "final_index_rows": 2}


@pytest.mark.parametrize("nb,m", [(1, 1), (5, 1), (7, 3), (9, 3), (10, 4)])
def test_all_distinct_closed_form(nb, m):
    bt = 64
    keys = datagen.key_of_rank(np.arange(nb * bt, dtype=np.uint64))
    r = spillsim.simulate(keys, batch_rows=bt, capacity=m * bt)
    runs = (nb - 1) // m
    assert r["runs"] == runs
    assert r["spilled_rows"] == runs * m * bt
    assert r["final_index_rows"] == (nb - runs * m) * bt


@pytest.mark.parametrize("s", [0.0, 0.8, 1.2])
def test_no_spill_when_output_fits(s):
    # Section 5 (no-spill table): the in-sort algorithm spills nothing when O <= M
    k, _, _ = datagen.plain_input(3, 50_000, 2_000, s)
    o = np.unique(k).shape[0]
    r = spillsim.simulate(k, batch_rows=1000, capacity=o)
    assert r["runs"] == 0 and r["spilled_rows"] == 0 and r["final_index_rows"] == o


def test_spill_bounded_by_input_and_model_shape():
    n, d = 200_000, 20_000
    k, _, _ = datagen.plain_input(4, n, d, 0.0)
    r = spillsim.simulate(k, batch_rows=500, capacity=5_000)
    assert 0 < r["spilled_rows"] <= n                               # each row spills at most once
    assert all(x <= 5_000 for x in r["run_sizes"])                  # runs never exceed memory
    o = np.unique(k).shape[0]
    model = spillsim.model_spill_rows(n, 5_000, o)
    assert 0.5 * model < r["spilled_rows"] < 1.5 * model            # same scale as the paper's model


def test_model_endpoints():
    # Section 3 Example 2: O = 2M gives M + I/2; O <= M gives no spill
    assert spillsim.model_spill_rows(1_000_000, 100_000, 200_000) == 100_000 + 500_000
    assert spillsim.model_spill_rows(1_000_000, 100_000, 100_000) == 0.0

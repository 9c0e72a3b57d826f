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


# ---------------------------------------------------------------------------
# Replacement selection through the index
# ---------------------------------------------------------------------------

def _classic_replacement_selection(keys, memory):
    """Textbook replacement selection with a priority queue of `memory` records
    tagged with their run: output the smallest key of the current run, read the
    next record into the freed slot, and tag it for the next run if it is below
    the key just written."""
    import heapq
    it = iter(int(x) for x in keys)
    heap = []
    for _ in range(memory):
        x = next(it, None)
        if x is None:
            break
        heap.append((0, x))
    heapq.heapify(heap)
    runs, cur = [], None
    while heap:
        r, x = heapq.heappop(heap)
        if r != cur:
            runs.append([])
            cur = r
        runs[-1].append(x)
        nxt = next(it, None)
        if nxt is not None:
            heapq.heappush(heap, (r if nxt >= x else r + 1, nxt))
    return runs


def test_replacement_hand_worked():
    # capacity 3, batches of 2 (worked by hand with the policy's steps):
    # {1,5}; {1,3,5,7} evicts 1; {2,3,5,7,9} evicts 2,3; {0,5,6,7,9} evicts
    # 5,6 (0 is below the cursor 4); {0,4,7,9,10} evicts 7,9; {0,4,8,10,11}
    # evicts 10,11; {0,2,3,4,8}: nothing at or after 12, so the run of 9 rows
    # ends and 0,2 start the next run
    r = spillsim.simulate_replacement([5, 1, 7, 3, 9, 2, 0, 6, 4, 10, 8, 11, 2, 3], 2, 3)
    assert r == {"runs": 2, "spilled_rows": 11, "run_sizes": [9, 2], "final_index_rows": 3}


@pytest.mark.parametrize("seed,n,K", [(1, 3000, 50), (2, 5000, 200), (3, 800, 7)])
def test_replacement_equals_priority_queue_with_one_row_batches(seed, n, K):
    # with batches of one row, evicting the smallest key at or after the
    # cursor from the index plus the new row is the textbook algorithm with
    # K + 1 slots, up to the point where the input ends (the index's last K
    # rows stay in memory)
    keys = np.random.default_rng(seed).permutation(10 * n)[:n].astype(np.uint64)
    r = spillsim.simulate_replacement(keys, 1, K)
    classic = _classic_replacement_selection(keys, K + 1)
    out = [x for run in classic for x in run][: n - K]
    sizes, left = [], n - K
    for run in classic:
        if left <= 0:
            break
        sizes.append(min(len(run), left))
        left -= len(run)
    assert r["spilled_rows"] == n - K == len(out)
    assert r["run_sizes"] == sizes


def test_replacement_sorted_input_makes_one_run():
    # the best case: ascending input never falls behind the scan
    n, K = 20_000, 1000
    r = spillsim.simulate_replacement(np.arange(n, dtype=np.uint64), 100, K)
    assert r["runs"] == 1 and r["spilled_rows"] == n - K


def test_replacement_descending_input_runs_are_memory_sized():
    # the worst case: every new key is below the scan, so each run holds one
    # memory load (K + 1 rows with one-row batches)
    n, K = 5000, 100
    r = spillsim.simulate_replacement(np.arange(n, 0, -1, dtype=np.uint64), 1, K)
    assert all(s == K + 1 for s in r["run_sizes"][:-1])
    assert r["spilled_rows"] == n - K


def test_replacement_random_runs_average_twice_memory():
    # random input: runs average about twice the memory (snowplow argument)
    n, K = 200_000, 2000
    keys = np.random.default_rng(7).permutation(n).astype(np.uint64)
    r = spillsim.simulate_replacement(keys, 1, K)
    full = r["run_sizes"][:-1]
    assert 1.85 * K <= np.mean(full) <= 2.15 * K, np.mean(full) / K


def test_replacement_no_spill_when_output_fits_and_never_more_runs():
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 500, 20_000).astype(np.uint64)
    r = spillsim.simulate_replacement(keys, 64, 500)
    assert r["runs"] == 0 and r["spilled_rows"] == 0
    # skewed input with duplicates: at most as many runs as read-sort-write,
    # the same final index size, spilled rows at most the input
    keys = rng.zipf(1.3, 60_000).astype(np.uint64)
    rs = spillsim.simulate_replacement(keys, 256, 2048)
    rw = spillsim.simulate(keys, 256, 2048)
    assert rs["runs"] <= rw["runs"] and rs["final_index_rows"] == 2048
    assert rs["spilled_rows"] <= keys.shape[0]


def test_preliminary_merges_example_4():
    # Section 4, Example 4: 500 runs of about 200,000 rows, fan-in 100, final
    # output 8,000,000 rows: the steps leave 496, 397, 298, 199 and 100 runs,
    # and the total spill volume is I + 1,000,000 + 4 x 8,000,000
    r = spillsim.preliminary_merges([200_000] * 500, 100, 8_000_000)
    assert r["counts"] == [500, 496, 397, 298, 199, 100]
    assert 100_000_000 + r["written_rows"] == 133_000_000


@pytest.mark.parametrize("n,F", [(1, 2), (7, 7), (8, 7), (13, 7), (100, 2), (376, 6), (1000, 100)])
def test_preliminary_merges_step_count(n, F):
    # ceil((n - F) / (F - 1)) steps, ending at exactly F runs (n > F), each
    # step after the first merging a full fan-in
    r = spillsim.preliminary_merges([1.0] * n, F, float("inf"))
    steps = max(0, -(-(n - F) // (F - 1)))
    assert len(r["counts"]) - 1 == steps
    assert r["counts"][-1] == (F if n > F else n)
    drops = [a - b for a, b in zip(r["counts"], r["counts"][1:])]
    assert all(d == F - 1 for d in drops[1:])
    # without an output bound the rows are conserved
    assert sum(r["final_runs"]) == n


def test_hybrid_plan_example():
    # Section 5's hybrid example: I = 275 M, F = 10, O = 2.75 M: f = 2, the
    # index holds 8/10 of memory and absorbs about 3/11 of the output, runs
    # store about 200 M rows in about 1,000 runs of 0.2 M, and one wide merge
    # suffices (O <= F M) where traditional merging needs 3 levels, 111 steps
    M = 100_000.0
    h = spillsim.hybrid_plan(275 * M, M, 2.75 * M, 10)
    assert h["f"] == 2
    assert abs(h["index_output_fraction"] - 0.8 / 2.75) < 1e-12
    # exactly 0.8/2.75 of the output: 195 M rows spill in 975 runs; the
    # paper rounds the fraction to 3/11, which gives its 200 M and 1,000
    assert abs(h["spilled_rows"] / M - 195.0) < 1e-6
    assert abs(h["run_rows"] - 0.2 * M) < 1e-9
    assert abs(h["runs"] - 975.0) < 1e-6
    assert abs(275 * (1 - 3 / 11) - 200.0) < 1e-9
    assert abs(275 * (1 - 3 / 11) * M / h["run_rows"] - 1000.0) < 1e-6
    assert h["single_wide_merge"]
    assert spillsim.traditional_levels(1000, 10) == (3, 111)


@pytest.mark.parametrize("O_over_M", [0.5, 1.0])
def test_hybrid_plan_in_memory_case(O_over_M):
    # O <= M: no fan-out, nothing spills
    h = spillsim.hybrid_plan(1e9, 1e5, O_over_M * 1e5, 10)
    assert h["f"] == 0 and h["spilled_rows"] == 0.0 and h["runs"] == 0.0


def test_preliminary_merges_exact_on_disjoint_runs_follows_the_plan():
    # runs with disjoint keys: every merge writes the sum of its inputs, so the
    # exact steps reproduce the size-only plan (Example 4's counts)
    rng = np.random.default_rng(3)
    keys = rng.permutation(500 * 40).astype(np.uint64)
    runs = [np.sort(keys[i * 40:(i + 1) * 40]) for i in range(500)]
    ex = spillsim.preliminary_merges_exact(runs, 100)
    plan = spillsim.preliminary_merges([40] * 500, 100, float("inf"))
    assert ex["counts"] == plan["counts"] == [500, 496, 397, 298, 199, 100]
    assert ex["written_rows"] == plan["written_rows"]
    assert sum(ex["final_run_sizes"]) == 500 * 40


def test_preliminary_merges_exact_combines_equal_keys():
    # hand-worked: fan-in 2 over runs {1,2}, {2,3,4}, {1,5}, {9}: each step
    # takes 2 runs, the smallest: {9} (1 row) and {1,2} (2 rows, written
    # before {1,5}) -> {1,2,9}; then {1,5} (2 rows) and {2,3,4} (3 rows,
    # written before {1,2,9} of the same size) -> {1,2,3,4,5}
    runs = [np.array([1, 2]), np.array([2, 3, 4]), np.array([1, 5]), np.array([9])]
    ex = spillsim.preliminary_merges_exact(runs, 2)
    assert ex["counts"] == [4, 3, 2]
    assert ex["step_rows"] == [3, 5]
    assert ex["final_run_sizes"] == [3, 5]


def test_simulate_keeps_run_keys():
    keys = np.array([5, 1, 5, 2, 7, 8, 9, 1, 3, 4], dtype=np.uint64)
    sim = spillsim.simulate(keys, 2, 3, keep_runs=True)
    assert [r.shape[0] for r in sim["run_keys"]] == sim["run_sizes"]
    for r in sim["run_keys"]:
        assert (np.diff(r.astype(np.int64)) > 0).all()
    # every key is in a run or in the final index; runs hold each key once
    seen = np.concatenate(sim["run_keys"]) if sim["run_keys"] else np.empty(0, np.uint64)
    assert seen.shape[0] == sim["spilled_rows"]


def test_hybrid_without_a_resident_index_is_read_sort_write():
    # no memory for the resident index (f = F): every key goes to runs, and
    # the runs are those of read-sort-write cycles
    k = datagen.plain_input(21, 60_000, 9_000, 0.5)[0]
    h = spillsim.simulate_hybrid(k, 1_000, 0, 3_000)
    r = spillsim.simulate(k, 1_000, 3_000)
    assert h["runs"] == r["runs"] and h["run_sizes"] == r["run_sizes"]
    assert h["resident_rows"] == 0 and h["final_index_rows"] == r["final_index_rows"]


def test_hybrid_output_fits_the_resident_index():
    # O <= resident capacity (f = 0): in-memory duplicate removal, no run
    k = datagen.plain_input(22, 50_000, 2_000, 0.0)[0]
    h = spillsim.simulate_hybrid(k, 1_000, 4_000, 1_000)
    assert h["runs"] == 0 and h["spilled_rows"] == 0
    assert h["resident_rows"] == np.unique(k).shape[0] and h["cut"] == 1 << 64


def test_hybrid_hand_worked():
    # batches of 2 rows, resident capacity 4 (keeps 3), run capacity 2
    keys = np.array([10, 20, 30, 40, 50, 5, 60, 70, 35, 80], dtype=np.uint64)
    h = spillsim.simulate_hybrid(keys, 2, 4, 2)
    # b1 {10,20} -> R {10,20}; b2 {30,40} -> R {10,20,30,40}; b3 {5,50} ->
    # R {5,10,20,30,40,50}: 6 > 4, demote {30,40,50}, cut 30, R {5,10,20};
    # b4 {60,70} -> gen {60,70}; b5 {35,80} -> gen {35,60,70,80} > 2: run
    # {60,70}, gen {35,80}
    assert h["run_sizes"] == [3, 2] and h["run_kinds"] == ["demotion", "run"]
    assert h["cut"] == 30 and h["resident_rows"] == 3 and h["final_index_rows"] == 5


def test_hybrid_scale_of_the_model():
    # Section 5's example scaled down: M = 10,000 rows, F = 10, O = 2.75 M,
    # I = 100 O, f = 2: an index of 8/10 of memory and runs from the other
    # 2/10.  The resident index keeps 3/4 of its capacity after a demotion,
    # so it absorbs 0.75 * 8,000 of the output's keys for good; the spilled
    # rows approach (1 - 6,000 / 27,500) of the input, less the duplicates
    # each run absorbs (about 5% for runs of 2,000 of the remaining ~21,500
    # keys: -D ln(1 - 2,000 / D) rows per run of 2,000 keys)
    M, O = 10_000, 27_500
    I = 100 * O
    h0 = spillsim.hybrid_plan(I, M, O, 10)
    assert h0["f"] == 2
    k = datagen.plain_input(23, I, O, 0.0)[0]
    Kr, Kw = int((1 - h0["f"] / 10) * M), int(h0["f"] / 10 * M)
    h = spillsim.simulate_hybrid(k, 500, Kr, Kw)
    D = O - 0.75 * Kr
    absorb = 1.0 - Kw / (-D * np.log(1 - Kw / D))
    expect = (1 - 0.75 * Kr / O) * I * (1 - absorb)
    assert abs(h["spilled_rows"] - expect) <= 0.05 * expect, (h["spilled_rows"], expect)
    assert h["spilled_rows"] < I
    assert abs(h["resident_rows"] - 0.75 * Kr) <= 0.25 * Kr


def test_absorb_first_hand_worked():
    # batches of 2 rows, capacity 3: {5,1} -> index {1,5}; {5,2} -> {1,2,5};
    # {7,8} -> {1,2,5,7,8} > 3: written whole (5 rows), index empty;
    # {9,1} -> {1,9}; {3,4} -> {1,3,4,9} > 3: written (4 rows), index empty
    keys = np.array([5, 1, 5, 2, 7, 8, 9, 1, 3, 4], dtype=np.uint64)
    r = spillsim.simulate(keys, 2, 3, absorb_first=True)
    assert r["run_sizes"] == [5, 4] and r["final_index_rows"] == 0


@pytest.mark.parametrize("nb,m", [(1000, 3), (700, 5), (512, 2)])
def test_absorb_first_all_distinct_closed_form(nb, m):
    # all keys distinct: the index grows by a batch until it holds more than
    # m batches, then (m + 1) batches are written: runs of (m + 1) * Bt rows
    n = nb * (m + 1) * 7 + nb * 2
    keys = datagen.key_of_rank(np.arange(n, dtype=np.uint64))
    r = spillsim.simulate(keys, nb, m * nb, absorb_first=True)
    assert r["run_sizes"] == [(m + 1) * nb] * 7
    assert r["final_index_rows"] == 2 * nb


@pytest.mark.parametrize("s", [0.0, 0.8, 1.2])
def test_absorb_first_bounds(s):
    # no run while the output fits the capacity; runs never exceed capacity
    # plus a batch, and spilled rows never exceed the input rows; the index
    # after a run starts empty, so each run holds more than capacity keys
    k = datagen.plain_input(31, 200_000, 20_000, s)[0]
    o = np.unique(k).shape[0]
    assert spillsim.simulate(k, 1_000, o, absorb_first=True)["runs"] == 0
    r = spillsim.simulate(k, 1_000, 4_000, absorb_first=True)
    assert all(4_000 < x <= 5_000 for x in r["run_sizes"])
    assert r["spilled_rows"] <= k.shape[0]
    sim_old = spillsim.simulate(k, 1_000, 4_000)
    # writing the memory whole as soon as it is full: about as many rows per
    # run as the other reading with one batch more of memory
    assert r["runs"] <= sim_old["runs"]

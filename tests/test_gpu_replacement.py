"""Replacement selection through the index (Section 3) on the GPU: output
against the oracle (integers bit-exact, fp64 within 1e-12 * sum |x|), and the
run count and spilled rows against the replacement-selection simulator with
the call's batch size and index capacity."""
import numpy as np
import pytest

import datagen
from oracle import spillsim
import paper_2010_00152_amd as isa
from tests.gpu_util import compare, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = isa.Context(0)
    c.set_run_generation(isa.ISA_RUNGEN_REPLACEMENT)
    yield c
    c.close()


def check_sim(k, st):
    sim = spillsim.simulate_replacement(k, st["batch_rows"], st["index_capacity"])
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    return sim


@pytest.mark.parametrize("s,seed,budget_mib", [(0.0, 5, 16), (0.8, 6, 16), (1.2, 7, 14), (0.5, 9, 24)])
def test_replacement_matches_oracle_and_simulator(ctx, s, seed, budget_mib):
    say("case replacement s=%s budget=%dMiB" % (s, budget_mib))
    n = 1_500_000
    k, v, f = datagen.plain_input(seed, n, 400_000, s, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=budget_mib << 20)
    compare(got, k, v, f, isa.ISA_ALL, "replacement")
    check_sim(k, st)
    if s < 1.2:
        assert st["runs"] > 0 and st["windows"] >= 1
    assert st["peak_ws_bytes"] <= budget_mib << 20


def test_replacement_sorted_input_one_run(ctx):
    # ascending distinct keys never fall behind the scan: one run
    say("case replacement sorted input")
    n = 2_000_000
    k = datagen.key_of_rank(np.arange(n, dtype=np.uint64))
    k = np.sort(k)
    v = datagen.uniform_i64(41, n)
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "sorted")
    assert st["runs"] == 1 and st["spilled_rows"] == n - st["index_capacity"]
    check_sim(k, st)


def test_replacement_descending_input(ctx):
    # descending distinct keys: every key lands below the scan (runs of one
    # index plus one batch).  The final index stays full under replacement
    # selection, so the wide merge needs a larger budget than read-sort-write.
    say("case replacement descending input")
    n = 2_000_000
    k = np.sort(datagen.key_of_rank(np.arange(n, dtype=np.uint64)))[::-1].copy()
    v = datagen.uniform_i64(42, n)
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=24 << 20)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "descending")
    sim = check_sim(k, st)
    assert st["runs"] >= 2 and max(sim["run_sizes"]) <= 2 * st["index_capacity"]


@pytest.mark.parametrize("aggs", [0, isa.ISA_COUNT, isa.ISA_SUM_F64])
def test_replacement_aggregate_subsets(ctx, aggs):
    say("case replacement aggs=%d" % aggs)
    k, v, f = datagen.plain_input(43, 1_800_000, 600_000, 0.3, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, aggs=aggs, budget=20 << 20)
    compare(got, k, v, f, aggs, "subset")
    assert st["runs"] > 0
    check_sim(k, st)


@pytest.mark.parametrize("budget_mib,force,extra", [(14, "0", 0), (14, "1", 1)])
def test_replacement_small_workspace_spills_the_final_index(ctx, monkeypatch, budget_mib, force, extra):
    # the final index stays full under replacement selection; when the rest
    # of the workspace cannot stage a wide merge beside it, the index is
    # written out as one more run and the merge reads host memory alone.
    # At 14 MiB the room suffices (no extra run); the rule's other side is
    # reached with ISA_FORCE_INDEX_SPILL=1, which treats the room as too
    # small (exactly one extra run holding the final index).  The
    # expected extra run is fixed per case, not read back from the result.
    say("case replacement workspace %d MiB force=%s" % (budget_mib, force))
    monkeypatch.setenv("ISA_FORCE_INDEX_SPILL", force)
    k, v, f = datagen.plain_input(43, 900_000, 300_000, 0.3, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, aggs=isa.ISA_SUM_F64, budget=budget_mib << 20)
    compare(got, k, v, f, isa.ISA_SUM_F64, "small")
    sim = spillsim.simulate_replacement(k, st["batch_rows"], st["index_capacity"])
    assert sim["runs"] > 0 and sim["final_index_rows"] > 0
    assert st["runs"] == sim["runs"] + extra, (st, sim)
    assert st["spilled_rows"] == sim["spilled_rows"] + extra * sim["final_index_rows"], (st, sim)


def test_replacement_same_output_as_read_sort_write(ctx):
    # the policy changes runs and spill volume, never the integer output; with
    # random input it needs fewer runs
    say("case replacement vs read-sort-write")
    k, v, _ = datagen.plain_input(44, 1_200_000, 600_000, 0.0)
    got_rs, st_rs, _, g_rs = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20)
    assert ctx.get_run_generation() == isa.ISA_RUNGEN_REPLACEMENT
    ctx.set_run_generation(isa.ISA_RUNGEN_READ_SORT_WRITE)
    try:
        got_w, st_w, _, g_w = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20)
    finally:
        ctx.set_run_generation(isa.ISA_RUNGEN_REPLACEMENT)
    assert g_rs == g_w
    for c in got_w:
        assert np.array_equal(got_rs[c], got_w[c]), c
    assert 0 < st_rs["runs"] < st_w["runs"]
    with pytest.raises(isa.InsortError):
        ctx.set_run_generation(7)

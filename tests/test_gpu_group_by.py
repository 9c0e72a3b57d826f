"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs, element by element.  Integer columns are bit-exact; the
fp64 sum is within 1e-12 * sum(|x|) per group."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import spillsim
import paper_2010_00152_amd as isa
from tests.gpu_util import compare, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = isa.Context(0)
    yield c
    c.close()


def test_plain_config_1m_rows_10k_keys(ctx):
    # plain group-by: 1M rows, uint64 keys uniform over 10,000 distinct values,
    # int64 values uniform in [-1e6, 1e6]; count/sum/min/max; budget above the output
    say("case plain 1M/10k seed 1")
    k, v, _ = datagen.plain_input(1, 1_000_000, 10_000, 0.0)
    aggs = isa.ISA_INT_AGGS
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=aggs, budget=64 << 20)
    assert status == isa.ISA_OK and st["runs"] == 0 and st["spilled_rows"] == 0
    compare(got, k, v, None, aggs, "plain")


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 4095, 4096, 4097, 16383, 16384, 16385, 65537, 300001])
def test_ragged_sizes(ctx, n):
    say("case ragged n=%d" % n)
    k, v, f = datagen.plain_input(100 + n % 97, n, max(1, n // 3), 0.7, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=64 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "ragged %d" % n)


def test_empty(ctx):
    say("case empty")
    import torch
    e = torch.empty(0, dtype=torch.int64, device="cuda")
    res, st, status, g = isa.group_by(ctx, e, e, torch.empty(0, dtype=torch.float64, device="cuda"),
                                      mem_budget=32 << 20, capacity=0)
    assert status == isa.ISA_OK and g == 0


@pytest.mark.parametrize("n", [4097, 200_000, 1_000_003])
def test_single_key(ctx, n):
    say("case single key n=%d" % n)
    k = np.full(n, 0x0123456789ABCDEF, np.uint64)
    v = datagen.uniform_i64(7, n)
    f = datagen.normal_f64(8, n)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=128 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "single")


def test_all_distinct(ctx):
    say("case all distinct")
    n = 300_000
    k = datagen.key_of_rank(np.arange(n, dtype=np.uint64) * np.uint64(7919))
    v = datagen.uniform_i64(9, n)
    f = datagen.normal_f64(10, n)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=128 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "distinct")


def test_extreme_keys_and_values(ctx):
    say("case extremes")
    n = 50_000
    rng = np.random.default_rng(3)
    pool = np.array([0, 1, 2, (1 << 63) - 1, 1 << 63, (1 << 64) - 2, (1 << 64) - 1], np.uint64)
    k = pool[rng.integers(0, len(pool), n)]
    vals = np.array([np.iinfo(np.int64).min, np.iinfo(np.int64).max, 0, -1, 1], np.int64)
    v = vals[rng.integers(0, len(vals), n)]
    f = rng.standard_normal(n) * 1e300
    got, st, status, g = run_gpu(ctx, k, v, f, budget=64 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "extremes")


@pytest.mark.parametrize("s,seed", [(0.0, 2), (0.8, 3), (1.2, 4)])
def test_zipf_all_aggs(ctx, s, seed):
    # the spilling configuration's shape at 1/50 scale, with a budget that holds it
    say("case zipf s=%s" % s)
    k, v, f = datagen.plain_input(seed, 2_000_000, 200_000, s, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=512 << 20)
    assert st["runs"] == 0
    compare(got, k, v, f, isa.ISA_ALL, "zipf %s" % s)


@pytest.mark.parametrize("s,seed,budget_mib", [(0.0, 5, 16), (0.8, 6, 16), (1.2, 7, 14), (0.0, 8, 24)])
def test_spilling_matches_oracle_and_simulator(ctx, s, seed, budget_mib):
    # a budget far below the output forces runs on pinned host memory and a
    # wide merge; the run count and spilled rows equal the read-sort-write
    # simulation with the same batch size and index capacity
    say("case spill s=%s budget=%dMiB" % (s, budget_mib))
    n = 1_500_000
    k, v, f = datagen.plain_input(seed, n, 400_000, s, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=budget_mib << 20)
    compare(got, k, v, f, isa.ISA_ALL, "spill")
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=True)
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    assert st["spilled_rows"] <= n
    if s < 1.2:
        assert st["runs"] > 0 and st["windows"] >= 1
    assert st["peak_ws_bytes"] <= budget_mib << 20


def test_budget_invariance(ctx):
    # integer output is independent of the budget (and so of batches, runs and windows)
    say("case budget invariance")
    k, v, _ = datagen.plain_input(12, 800_000, 150_000, 0.5)
    outs = []
    for b in [16 << 20, 40 << 20, 512 << 20]:
        got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=b)
        outs.append(got)
    for o in outs[1:]:
        for c in o:
            assert np.array_equal(o[c], outs[0][c]), c


@pytest.mark.parametrize("aggs", [0, isa.ISA_COUNT, isa.ISA_SUM_F64, isa.ISA_MIN_I64,
                                  isa.ISA_MAX_I64 | isa.ISA_SUM_I64])
def test_aggregate_subsets(ctx, aggs):
    say("case aggs=%d" % aggs)
    k, v, f = datagen.plain_input(13, 120_000, 20_000, 0.9, with_f64=True)
    vv = v if aggs & (isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64) else None
    ff = f if aggs & isa.ISA_SUM_F64 else None
    got, st, status, g = run_gpu(ctx, k, vv, ff, aggs=aggs, budget=64 << 20)
    compare(got, k, vv, ff, aggs, "aggs %d" % aggs)


def test_truncation(ctx):
    say("case truncation")
    k, v, _ = datagen.plain_input(14, 100_000, 5_000, 0.0)
    ref = oracle.group_by(k, v)
    G = ref["keys"].shape[0]
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=64 << 20,
                                 capacity=G - 7, check=False)
    assert status == isa.ISA_ETRUNC and g == G
    assert np.array_equal(got["keys"], ref["keys"][:G - 7])
    assert np.array_equal(got["sum_i64"], ref["sum_i64"][:G - 7])


def test_argument_errors(ctx):
    say("case argument errors")
    import torch
    k, v, f = datagen.plain_input(15, 10_000, 100, 0.0, with_f64=True)
    kd = torch.from_numpy(k.view(np.int64)).cuda()
    # a requested aggregate without its column
    with pytest.raises(isa.InsortError) as e:
        isa.group_by(ctx, kd, None, None, aggs=isa.ISA_SUM_I64, mem_budget=32 << 20)
    assert e.value.status == isa.ISA_EINVAL
    # workspace below the minimum
    with pytest.raises(isa.InsortError) as e:
        isa.group_by(ctx, kd, None, None, aggs=isa.ISA_COUNT, mem_budget=1 << 20)
    assert e.value.status == isa.ISA_EBUDGET
    # no room to spill
    k2, v2, _ = datagen.plain_input(16, 1_000_000, 500_000, 0.0)
    kd2 = torch.from_numpy(k2.view(np.int64)).cuda()
    vd2 = torch.from_numpy(v2).cuda()
    with pytest.raises(isa.InsortError) as e:
        isa.group_by(ctx, kd2, vd2, None, aggs=isa.ISA_INT_AGGS, mem_budget=16 << 20, spill_bytes=0)
    assert e.value.status == isa.ISA_ESPILL


@pytest.mark.parametrize("n", [100, 3000, 4095])
def test_leaf_max_key_ties_with_padding(ctx, n):
    # a leaf smaller than the workgroup tile: rows holding the leaf's largest
    # key must sort before the padding rows that share that key value
    say("case max-key ties n=%d" % n)
    rng = np.random.default_rng(n)
    k = rng.integers(0, 50, n).astype(np.uint64)
    k[rng.random(n) < 0.4] = np.uint64(49)
    v = rng.integers(-1000, 1000, n).astype(np.int64)
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=32 << 20)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "ties %d" % n)


# Keys in clusters: every key of a cluster is its centre plus a low part
# below 2^20, and centres are multiples of 2^51, so within any leaf the keys
# of one cluster agree on every bit a leaf sorts before its clash fix-up
# (the top 24 or so bits of the leaf's key range) and differ only below.
# Cases: a few short clusters in one leaf (ranked in place), clusters longer
# than the fix-up takes, more clusters than it takes (both re-sorted at full
# width), and a 200K-row input whose buckets each hold several clusters (the
# single-level plan's leaves).  Low parts repeat, so groups have many rows.
@pytest.mark.parametrize("n, clusters, pool", [(3000, 8, 200), (3500, 2, 100_000), (3000, 40, 40),
                                               (4096, 32, 2000), (200_000, 2000, 60)])
def test_leaf_key_clashes(ctx, n, clusters, pool):
    say("case clashes n=%d clusters=%d pool=%d" % (n, clusters, pool))
    rng = np.random.default_rng(n + clusters)
    centres = np.sort(rng.choice(1 << 13, clusters, replace=False)).astype(np.uint64) << np.uint64(51)
    lows = rng.integers(0, 1 << 20, size=(clusters, pool)).astype(np.uint64)
    c = rng.integers(0, clusters, n)
    k = centres[c] + lows[c, rng.integers(0, pool, n)]
    v = rng.integers(-(1 << 40), 1 << 40, n).astype(np.int64)
    f = rng.standard_normal(n)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=256 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "clashes %d/%d" % (n, clusters))


def test_flat_plan_falls_back_on_oversized_bucket(ctx):
    # every row the splitter sample reads holds the same key, all other rows
    # are distinct: the sampled splitters isolate that key and leave two huge
    # multi-key buckets, which the single-level plan cannot take; the call must
    # still give the exact result (through the multi-level plan)
    say("case flat fallback")
    n, S = 300_000, 4096
    k = datagen.key_of_rank(np.arange(n, dtype=np.uint64) + np.uint64(10))
    pos = ((2 * np.arange(S, dtype=np.int64) + 1) * n) // (2 * S)
    k[pos] = np.uint64(1 << 62)
    v = datagen.uniform_i64(17, n)
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=128 << 20)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "fallback")


def test_spilling_with_extreme_keys(ctx):
    # runs whose first and last keys are 0 and 2^64-1: the wide merge's key
    # windows must end exactly at the largest key value
    say("case spill extreme keys")
    n = 900_000
    rng = np.random.default_rng(21)
    k, v, f = datagen.plain_input(22, n, 300_000, 0.0, with_f64=True)
    pool = np.array([0, 1, 1 << 63, (1 << 64) - 2, (1 << 64) - 1], np.uint64)
    pick = rng.random(n) < 0.3
    k = k.copy()
    k[pick] = pool[rng.integers(0, len(pool), int(pick.sum()))]
    got, st, status, g = run_gpu(ctx, k, v, f, budget=16 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "spill extremes")
    assert st["runs"] > 0
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=True)
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)


@pytest.mark.parametrize("aggs", [isa.ISA_ALL, isa.ISA_INT_AGGS, isa.ISA_COUNT | isa.ISA_SUM_F64,
                                  isa.ISA_COUNT | isa.ISA_MIN_I64])
def test_spilling_count1_value_widths(ctx, aggs):
    # a run's count-1 rows keep their integer values in 4 bytes when all of
    # them fit in 32 bits: the early batches hold only such values (the 32-bit
    # limits included), the later ones also values just outside them, so runs
    # of both widths meet in the wide merge
    say("case spill count-1 widths aggs=%d" % aggs)
    n = 1_200_000
    rng = np.random.default_rng(41)
    k, v, f = datagen.plain_input(42, n, 400_000, 0.5, with_f64=True)
    v = v.copy()
    lim = np.array([-(1 << 31), (1 << 31) - 1], np.int64)
    early = rng.random(n) < 0.05
    early[n * 3 // 5:] = False
    v[early] = lim[rng.integers(0, 2, int(early.sum()))]
    late = rng.random(n) < 0.05
    late[:n * 3 // 5] = False
    out = np.array([-(1 << 31) - 1, 1 << 31, -(1 << 40), 1 << 40], np.int64)
    v[late] = out[rng.integers(0, 4, int(late.sum()))]
    vv = v if aggs & (isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64) else None
    ff = f if aggs & isa.ISA_SUM_F64 else None
    got, st, status, g = run_gpu(ctx, k, vv, ff, aggs=aggs, budget=16 << 20)
    assert status == isa.ISA_OK
    assert st["runs"] > 1
    compare(got, k, vv, ff, aggs, "count-1 widths")


def test_wide_merge_second_pass(ctx, monkeypatch):
    # the wide merge places every window's groups after a device-side cursor
    # and falls back to a host-paced second pass when a window's flat plan
    # fails; both passes must give the oracle's output
    say("case wide merge second pass")
    n = 900_000
    k, v, f = datagen.plain_input(31, n, 300_000, 0.8, with_f64=True)
    got1, st1, status1, g1 = run_gpu(ctx, k, v, f, budget=16 << 20)
    compare(got1, k, v, f, isa.ISA_ALL, "first pass")
    assert st1["runs"] > 0 and st1["windows"] > 1
    monkeypatch.setenv("ISA_FORCE_MERGE_REDO", "1")
    got2, st2, status2, g2 = run_gpu(ctx, k, v, f, budget=16 << 20)
    compare(got2, k, v, f, isa.ISA_ALL, "second pass")
    assert g2 == g1 and st2["windows"] == st1["windows"]
    for col in ("keys", "count", "sum_i64", "min_i64", "max_i64"):
        assert np.array_equal(got1[col], got2[col]), col


@pytest.mark.parametrize("redo", ["0", "1"])
def test_truncation_while_spilling(ctx, monkeypatch, redo):
    # an output capacity below the group count while the wide merge places
    # windows behind a device-side cursor (first pass) or a host cursor
    # (second pass): ETRUNC, the full group count, and the first rows exact
    say("case truncation while spilling redo=%s" % redo)
    monkeypatch.setenv("ISA_FORCE_MERGE_REDO", redo)
    k, v, _ = datagen.plain_input(16, 900_000, 300_000, 0.5)
    ref = oracle.group_by(k, v)
    G = ref["keys"].shape[0]
    for cap in (G // 3, G - 1234):
        got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20, capacity=cap,
                                     check=False)
        assert st["runs"] > 0 and st["windows"] > 1
        assert status == isa.ISA_ETRUNC and g == G
        for col in ("keys", "count", "sum_i64", "min_i64", "max_i64"):
            assert np.array_equal(got[col], ref[col][:cap]), (cap, col)


@pytest.mark.parametrize("fanin", [3, 4])
def test_preliminary_merges_before_the_wide_merge(ctx, fanin):
    # with a merge fan-in below the run count, the smallest runs are merged
    # first (Section 4, Example 4) so that the final wide merge takes at most
    # `fanin` runs; the output equals the oracle's, and the steps, the rows
    # they write and the runs left equal the exact simulation of the same plan.
    # Merged runs are state rows beside the compact initial runs, so the
    # temporary storage is sized above one state row per input row.
    say("case preliminary merges fan-in %d" % fanin)
    n = 1_500_000
    k, v, f = datagen.plain_input(5, n, 400_000, 0.0, with_f64=True)
    ctx.set_tuning(merge_fanin=fanin)
    try:
        got, st, status, g = run_gpu(ctx, k, v, f, budget=16 << 20, spill_bytes=3 * n * 48)
    finally:
        ctx.set_tuning()
    compare(got, k, v, f, isa.ISA_ALL, "preliminary merges")
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], keep_runs=True, absorb_first=True)
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    plan = spillsim.preliminary_merges_exact(sim["run_keys"], fanin)
    assert len(plan["counts"]) - 1 >= 2                     # at least two steps
    assert st["merge_steps"] == len(plan["counts"]) - 1, (st, plan["counts"])
    assert st["merge_rows"] == plan["written_rows"], (st, plan)
    assert st["windows"] >= 1


def test_inplace_runs_compacted_or_as_state_rows(ctx):
    # read-sort-write absorbs batches in place and compacts each run into a
    # spare area of about half the index; a run whose compacted form would not
    # fit (few count-1 rows, wide values) goes out as state rows instead.
    # Both give the oracle's output and the simulator's runs and rows.
    n = 1_200_000
    sw = 48
    # many count-1 rows and 32-bit values: every run compacted
    say("case in-place compacted runs")
    k, v, f = datagen.plain_input(51, n, 600_000, 0.0, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=16 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "in-place compacted")
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=True)
    assert st["runs"] == sim["runs"] > 1 and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    assert st["spilled_bytes"] < 0.6 * sw * st["spilled_rows"]
    # a key domain near the index capacity and 64-bit values: more than half
    # of each run's keys repeat, and no compacted run fits the spare area
    say("case in-place state-row runs")
    rng = np.random.default_rng(52)
    k = datagen.key_of_rank(rng.integers(0, 80_000, n).astype(np.uint64))
    v = rng.integers(-(1 << 40), 1 << 40, n).astype(np.int64)
    f = rng.standard_normal(n)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=16 << 20)
    compare(got, k, v, f, isa.ISA_ALL, "in-place state rows")
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=True)
    assert st["runs"] == sim["runs"] > 1 and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    assert st["spilled_bytes"] == sw * st["spilled_rows"]


@pytest.mark.parametrize("aggs", [0, isa.ISA_COUNT, isa.ISA_SUM_F64, isa.ISA_MIN_I64,
                                  isa.ISA_MAX_I64 | isa.ISA_SUM_I64, isa.ISA_COUNT | isa.ISA_SUM_F64])
def test_spilling_aggregate_subsets(ctx, aggs):
    # Aggregate sets without a count column write their runs as state rows
    # and keep two index buffers (the other batch-granular rule of R8); a
    # count with an f64 sum alone compacts its runs but keeps two buffers (its
    # raw row is more than half a state row); a count alone absorbs in place.
    # Every form: the oracle's output and the simulator's runs and rows.
    say("case spilling aggs=%d" % aggs)
    n = 1_200_000
    k, v, f = datagen.plain_input(61, n, 400_000, 0.4, with_f64=True)
    vv = v if aggs & (isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64) else None
    ff = f if aggs & isa.ISA_SUM_F64 else None
    got, st, status, g = run_gpu(ctx, k, vv, ff, aggs=aggs, budget=16 << 20)
    compare(got, k, vv, ff, aggs, "spilling aggs %d" % aggs)
    in_place = aggs in (isa.ISA_COUNT,)
    sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=in_place)
    assert st["runs"] == sim["runs"] > 0 and st["spilled_rows"] == sim["spilled_rows"], (aggs, st, sim)
    row_b = isa.lib().isa_state_row_bytes(aggs)
    if not aggs & isa.ISA_COUNT:
        assert st["spilled_bytes"] == row_b * st["spilled_rows"]      # state rows only
    else:
        assert st["spilled_bytes"] < row_b * st["spilled_rows"]       # compacted

"""GPU parity of the segmented, batched and served forms against the CPU
oracle, and equality of each instance's result alone and in a batch."""
import time

import numpy as np
import pytest

import datagen
import oracle
import paper_2010_00152_amd as isa
from tests.gpu_util import run_gpu, FP64_REL, compare, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = isa.Context(0)
    yield c
    c.close()


def np_out(res):
    out = {}
    for k, t in res.items():
        dt = {"keys": np.uint64, "count": np.uint64, "sum_f64": np.float64, "a": np.int32,
              "b": np.int32}.get(k, np.int64)
        out[k] = to_np(t, dt)
    return out


@pytest.mark.parametrize("n,n_a,b_per_a,budget_mib", [(300_000, 40, 3_000, 64), (2_000_000, 1000, 100_000, 64),
                                                      (3_000_000, 7, 400_000, 256)])
def test_segmented_matches_pair_oracle(ctx, n, n_a, b_per_a, budget_mib):
    say("case segmented n=%d n_a=%d" % (n, n_a))
    a, b, v = datagen.segmented_input(5, n, n_a, b_per_a)
    res, status, g = isa.group_by_segmented(ctx, to_dev(a), to_dev(b), to_dev(v), aggs=isa.ISA_INT_AGGS,
                                            mem_budget=budget_mib << 20)
    got = np_out(res)
    ref = oracle.group_by_pairs(a, b, v)
    assert g == ref["a"].shape[0]
    for c in ["a", "b", "count", "sum_i64", "min_i64", "max_i64"]:
        assert np.array_equal(got[c], ref[c]), c


# The waves of segments run back to back with device-side output rows by
# default; ISA_SEGMENTED_SYNC=1 takes the loop that waits for every wave, and
# a segment longer than the single-level plan takes (here 600K rows) sends
# the call there by itself.  Both must give the oracle's result, also when
# the output is truncated (the first rows, then ISA_ETRUNC).
@pytest.mark.parametrize("sync", [False, True])
@pytest.mark.parametrize("n,n_a,b_per_a,budget_mib,cap", [(2_000_000, 1000, 100_000, 32, None),
                                                          (1_200_000, 2, 100_000, 128, None),
                                                          (2_000_000, 1000, 100_000, 32, 700_000)])
def test_segmented_wave_loops(ctx, monkeypatch, sync, n, n_a, b_per_a, budget_mib, cap):
    say("case segmented waves sync=%d n=%d n_a=%d cap=%s" % (sync, n, n_a, cap))
    if sync:
        monkeypatch.setenv("ISA_SEGMENTED_SYNC", "1")
    a, b, v = datagen.segmented_input(9, n, n_a, b_per_a)
    res, status, g = isa.group_by_segmented(ctx, to_dev(a), to_dev(b), to_dev(v), aggs=isa.ISA_INT_AGGS,
                                            mem_budget=budget_mib << 20, capacity=cap, check=False)
    got = np_out(res)
    ref = oracle.group_by_pairs(a, b, v)
    G = ref["a"].shape[0]
    assert g == G
    m = G if cap is None else min(cap, G)
    assert status == (isa.ISA_ETRUNC if m < G else isa.ISA_OK)
    for c in ["a", "b", "count", "sum_i64", "min_i64", "max_i64"]:
        assert np.array_equal(got[c], ref[c][:m]), c


def test_segmented_flat_plan_failure_falls_back(ctx):
    # one 300K-row segment whose rows at the splitter sample's positions all
    # hold the same B value, all other B values distinct: the sampled
    # splitters isolate that value and leave two multi-key buckets far above
    # a leaf, the pipelined wave's flat plan reports it, and the call must
    # still give the exact result through the wave-at-a-time loop
    say("case segmented flat fallback")
    n, S = 300_000, 4096
    a = np.zeros(n, np.int32)
    b = (np.arange(n, dtype=np.int64) * 7919 % (1 << 30)).astype(np.int32)
    pos = ((2 * np.arange(S, dtype=np.int64) + 1) * n) // (2 * S)
    b[pos] = np.int32(123)
    v = datagen.uniform_i64(19, n)
    res, status, g = isa.group_by_segmented(ctx, to_dev(a), to_dev(b), to_dev(v), aggs=isa.ISA_INT_AGGS,
                                            mem_budget=128 << 20)
    got = np_out(res)
    ref = oracle.group_by_pairs(a, b, v)
    assert g == ref["a"].shape[0]
    for c in ["a", "b", "count", "sum_i64", "min_i64", "max_i64"]:
        assert np.array_equal(got[c], ref[c]), c


def test_segmented_rejects_unsorted_prefix(ctx):
    say("case segmented unsorted")
    a = np.array([1, 2, 1, 3] * 1000, np.int32)
    b = np.arange(4000, dtype=np.int32)
    v = np.zeros(4000, np.int64)
    with pytest.raises(isa.InsortError) as e:
        isa.group_by_segmented(ctx, to_dev(a), to_dev(b), to_dev(v), mem_budget=32 << 20)
    assert e.value.status == isa.ISA_EINVAL


def batch_instances(seed, count, lo, hi):
    rng = np.random.default_rng(seed)
    rows = np.exp(rng.uniform(np.log(lo), np.log(hi), count)).round().astype(np.int64)
    ratio = np.exp(rng.uniform(np.log(1e-4), 0.0, count))
    insts = []
    for i in range(count):
        d = max(1, int(round(rows[i] * ratio[i])))
        k, v, f = datagen.plain_input(datagen.substream_seed(seed, i), int(rows[i]), d, 0.0, with_f64=True)
        insts.append((k, v, f))
    return insts


def test_batch_matches_oracle_and_alone(ctx):
    say("case batch 300 instances")
    insts = batch_instances(6, 300, 1_000, 100_000)
    dev = [(to_dev(k), to_dev(v), to_dev(f)) for k, v, f in insts]
    res, status = isa.batch_run(ctx, dev, aggs=isa.ISA_ALL, mem_budget=512 << 20)
    for i, (k, v, f) in enumerate(insts):
        compare(np_out(res[i]), k, v, f, isa.ISA_ALL, "inst %d" % i)
    # alone: the same instance through the plain entry point gives identical integers
    for i in [0, 7, 150, 299]:
        k, v, f = insts[i]
        alone, st, _, _ = isa.group_by(ctx, dev[i][0], dev[i][1], dev[i][2], aggs=isa.ISA_ALL, mem_budget=64 << 20)
        a = np_out(alone)
        b = np_out(res[i])
        for c in ["keys", "count", "sum_i64", "min_i64", "max_i64"]:
            assert np.array_equal(a[c], b[c]), (i, c)
        absum = oracle.group_by(k, None, np.abs(f))["sum_f64"]
        assert np.all(np.abs(a["sum_f64"] - b["sum_f64"]) <= 2 * FP64_REL * absum)


def test_batch_waves_small_workspace(ctx):
    # a workspace that holds only a few instances at a time: processed in waves
    say("case batch waves")
    insts = batch_instances(16, 40, 20_000, 200_000)
    dev = [(to_dev(k), to_dev(v), None) for k, v, f in insts]
    res, status = isa.batch_run(ctx, dev, aggs=isa.ISA_INT_AGGS, mem_budget=48 << 20)
    for i, (k, v, f) in enumerate(insts):
        compare(np_out(res[i]), k, v, None, isa.ISA_INT_AGGS, "inst %d" % i)


@pytest.mark.parametrize("cfg", [dict(leaf_rows=1024, chunk_split=256, graph=1),
                                 dict(leaf_rows=1536, chunk_split=1024, graph=0),
                                 dict(leaf_rows=256, chunk_split=64, graph=1),
                                 dict(leaf_rows=2048, chunk_split=4096, graph=0)])
def test_tuning_changes_speed_not_results(ctx, cfg):
    # every launch configuration gives the oracle's result (I9), on the
    # batched path (flat plan, both size classes) and on the spilling path
    say("case tuning %r" % (cfg,))
    insts = batch_instances(26, 30, 1_000, 700_000)
    dev = [(to_dev(k), to_dev(v), None) for k, v, f in insts]
    ctx.set_tuning(**cfg)
    try:
        assert ctx.get_tuning() == dict(isa.Context.default_tuning(), **cfg)
        res, status = isa.batch_run(ctx, dev, aggs=isa.ISA_INT_AGGS, mem_budget=512 << 20)
        for i, (k, v, f) in enumerate(insts):
            compare(np_out(res[i]), k, v, None, isa.ISA_INT_AGGS, "inst %d" % i)
        k, v, f = datagen.plain_input(27, 1_200_000, 300_000, 0.8, with_f64=True)
        got, st, _, _ = run_gpu(ctx, k, v, f, budget=24 << 20)
        assert st["runs"] > 0
        compare(got, k, v, f, isa.ISA_ALL, "spill under tuning")
    finally:
        ctx.set_tuning()


def test_tuning_rejects_out_of_range(ctx):
    for bad in [dict(leaf_rows=100), dict(leaf_rows=4096), dict(chunk_split=8), dict(graph=2),
                dict(merge_fanin=1), dict(merge_fanin=65537)]:
        with pytest.raises(isa.InsortError) as e:
            ctx.set_tuning(**bad)
        assert e.value.status == isa.ISA_EINVAL
    assert ctx.get_tuning() == isa.Context.default_tuning()


def test_autotuner_picks_a_candidate_and_keeps_results(ctx):
    say("case autotuner")
    insts = batch_instances(28, 40, 1_000, 200_000)
    dev = [(to_dev(k), to_dev(v), None) for k, v, f in insts]
    best, times = isa.tune_batch(ctx, dev, aggs=isa.ISA_INT_AGGS, mem_budget=512 << 20)
    cands = isa.tune_candidates()
    assert best in cands and len(times) == len(cands) and all(t > 0 for t in times.values())
    assert ctx.get_tuning() == best
    assert times[cands.index(best)] == min(times.values())
    res, status = isa.batch_run(ctx, dev, aggs=isa.ISA_INT_AGGS, mem_budget=512 << 20)
    for i, (k, v, f) in enumerate(insts):
        compare(np_out(res[i]), k, v, None, isa.ISA_INT_AGGS, "inst %d" % i)
    ctx.set_tuning()


def test_server_results_alone_and_in_the_mix(ctx):
    # 60 requests of different sizes arrive while others run (3 slots, so
    # their device work overlaps); every result matches the oracle, and a
    # subset run again alone (a one-slot server with one request in flight)
    # gives the same result as in the mix: integers bit-equal, the fp64 sum
    # within 1e-12 * sum |x|
    say("case server")
    import torch
    insts = batch_instances(7, 60, 1_000, 300_000)
    dev = [(to_dev(k), to_dev(v), to_dev(f)) for k, v, f in insts]
    torch.cuda.synchronize()
    srv = isa.Server(ctx, 1 << 30, slots=3)
    tickets = []
    for i, (k, v, f) in enumerate(dev):
        tickets.append(srv.submit(k, v, f, aggs=isa.ISA_ALL))
        if i % 7 == 0:
            time.sleep(0.002)  # requests keep arriving while others run
    srv.drain()
    mix = {}
    for i, t in enumerate(tickets):
        done, lat, st = srv.poll(t)
        assert done and st == isa.ISA_OK and lat > 0
        k, v, f = insts[i]
        mix[i] = np_out(srv.release(t))
        compare(mix[i], k, v, f, isa.ISA_ALL, "req %d" % i)
        assert srv.poll(t)[2] == isa.ISA_EINVAL        # a released ticket is unknown
    assert not srv.live
    srv.close()

    alone = isa.Server(ctx, 1 << 30, slots=1)
    for i in range(0, len(insts), 4):
        k, v, f = dev[i]
        t = alone.submit(k, v, f, aggs=isa.ISA_ALL)
        alone.drain()
        done, lat, st = alone.poll(t)
        assert done and st == isa.ISA_OK
        got = np_out(alone.release(t))
        for col in ("keys", "count", "sum_i64", "min_i64", "max_i64"):
            assert np.array_equal(got[col], mix[i][col]), (i, col)
        absum = oracle.group_by(insts[i][0], None, np.abs(insts[i][2]))["sum_f64"]
        assert (np.abs(got["sum_f64"] - mix[i]["sum_f64"]) <= FP64_REL * absum).all(), i
    alone.close()


def test_server_rejects_oversized_request(ctx):
    say("case server oversized")
    import torch
    srv = isa.Server(ctx, 32 << 20, slots=1)
    k = torch.zeros(2_000_000, dtype=torch.int64, device="cuda")
    with pytest.raises(isa.InsortError) as e:
        srv.submit(k, k, None, aggs=isa.ISA_INT_AGGS)
    assert e.value.status == isa.ISA_ENOMEM
    srv.close()

"""Parity at full size, in the launch configuration the benchmark times.

* Spilling group-by: 100M rows, uint64 keys over 1e7 Zipf(s) ranks for s in
  {0, 0.8, 1.2}, int64 and float64 values, all aggregates, 256 MiB workspace
  and a pinned spill buffer (runs and a wide merge); at s = 0.8 also with run
  generation by replacement selection.
* Segmented grouping: 200M rows, (A, B) int32 with 1e3 A values and 1e5 B
  values per A, sorted on A only, 256 MiB workspace.
* One wave of the batched configuration (every instance of the wave).

Every output row of every column is compared with the oracle run on the whole
input (the oracle's sort-then-scan plan on up to 16 host threads over key
ranges, bit-identical to its single-threaded form): integers bit-exact, the
fp64 sum within 1e-12 * sum |x| per group.  The invariants (strictly
increasing keys, total count, int64 sum mod 2^64, global min and max) are
checked as well.  Spill statistics equal the simulator's for the call's
run-generation policy.  Each case prints its oracle time.
"""
import time

import numpy as np
import pytest

import oracle
from oracle import spillsim
import paper_2010_00152_amd as isa
from tests.gpu_util import FP64_REL, say, to_np

# host threads of the oracle: the machine's CPU share, whatever nproc reports
ORACLE_THREADS = 16

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = isa.Context(0)
    yield c
    c.close()


def _host(res):
    out = {}
    for k, t in res.items():
        dt = {"keys": np.uint64, "count": np.uint64, "sum_f64": np.float64, "a": np.int32,
              "b": np.int32}.get(k, np.int64)
        out[k] = to_np(t, dt)
    return out


@pytest.mark.timeout(900)
@pytest.mark.parametrize("s,seed,policy", [(0.0, 2, "rsw"), (0.8, 3, "rsw"), (1.2, 4, "rsw"), (0.8, 3, "rs")])
def test_spilling_100m_rows_full_size(ctx, s, seed, policy):
    import torch
    import datagen.device as dgd
    n, d = 100_000_000, 10_000_000
    say("case full-size spill n=%d d=%d s=%s seed=%d policy=%s" % (n, d, s, seed, policy))
    kd, vd, fd = dgd.plain_input(seed, n, d, s, with_f64=True)
    ctx.set_run_generation(isa.ISA_RUNGEN_REPLACEMENT if policy == "rs" else isa.ISA_RUNGEN_READ_SORT_WRITE)
    try:
        res, st, status, g = isa.group_by(ctx, kd, vd, fd, aggs=isa.ISA_ALL, mem_budget=256 << 20,
                                          capacity=min(n, d))
    finally:
        ctx.set_run_generation(isa.ISA_RUNGEN_READ_SORT_WRITE)
    torch.cuda.synchronize()
    say("  groups %d runs %d spilled %d windows %d" % (g, st["runs"], st["spilled_rows"], st["windows"]))
    got = _host(res)
    k, v, f = to_np(kd, np.uint64), to_np(vd, np.int64), to_np(fd, np.float64)
    del kd, vd, fd, res

    keys = got["keys"]
    assert keys.shape[0] == g
    assert (keys[1:] > keys[:-1]).all()                       # sorted, unique
    assert int(got["count"].sum()) == n
    assert got["sum_i64"].sum() == v.sum()                    # mod 2^64 on both sides
    assert got["min_i64"].min() == v.min() and got["max_i64"].max() == v.max()

    t0 = time.time()
    threads = min(ORACLE_THREADS, oracle.nproc())
    ref = oracle.group_by(k, v, f, threads=threads)
    absum = oracle.group_by(k, None, np.abs(f), threads=threads)["sum_f64"]
    say("  oracle on the whole input: %.1f s (%d threads)" % (time.time() - t0, threads))
    assert np.array_equal(keys, ref["keys"])
    for col in ("count", "sum_i64", "min_i64", "max_i64"):
        assert np.array_equal(got[col], ref[col]), col
    err = np.abs(got["sum_f64"] - ref["sum_f64"])
    bad = err > FP64_REL * absum
    assert not bad.any(), (int(bad.sum()), float((err / np.maximum(absum, 1e-300)).max()))
    del ref, absum, err

    if policy == "rs":
        sim = spillsim.simulate_replacement(k, st["batch_rows"], st["index_capacity"])
    else:
        sim = spillsim.simulate(k, st["batch_rows"], st["index_capacity"], absorb_first=True)
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    assert st["spilled_rows"] <= n
    assert st["peak_ws_bytes"] <= 256 << 20
    if s < 1.0:
        assert st["runs"] > 0 and st["windows"] > 0             # the budget forces runs and a wide merge


@pytest.mark.timeout(900)
def test_segmented_200m_rows_full_size(ctx):
    import torch
    import datagen.device as dgd
    n = 200_000_000
    say("case full-size segmented n=%d seed=5" % n)
    ad, bd, vd = dgd.segmented_input(5, n)
    res, status, g = isa.group_by_segmented(ctx, ad, bd, vd, aggs=isa.ISA_INT_AGGS, mem_budget=256 << 20)
    torch.cuda.synchronize()
    say("  groups %d" % g)
    got = _host(res)
    a, b, v = to_np(ad, np.int32), to_np(bd, np.int32), to_np(vd, np.int64)
    del ad, bd, vd, res

    def packed(x, y):
        # (A, B) in signed lexicographic order as one unsigned key
        return ((x.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64) << np.uint64(32)) | \
            (y.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64)

    assert (a[1:] >= a[:-1]).all()
    pk = packed(got["a"], got["b"])
    assert pk.shape[0] == g and (pk[1:] > pk[:-1]).all()
    assert got["sum_i64"].sum() == v.sum()
    assert got["min_i64"].min() == v.min() and got["max_i64"].max() == v.max()
    # every group through the oracle: the pair (A, B) as one normalized key
    # (the 24 segments below check that ordering against the pair oracle)
    t0 = time.time()
    threads = min(ORACLE_THREADS, oracle.nproc())
    ref = oracle.group_by(packed(a, b), v, None, threads=threads)
    say("  oracle on the whole input: %.1f s (%d threads)" % (time.time() - t0, threads))
    assert np.array_equal(pk, ref["keys"])
    for col in ("count", "sum_i64", "min_i64", "max_i64"):
        assert np.array_equal(got[col], ref[col]), col
    del ref

    seg_vals = np.unique(a)
    rng = np.random.default_rng(55)
    for av in rng.choice(seg_vals, size=24, replace=False):
        lo, hi = np.searchsorted(a, av, "left"), np.searchsorted(a, av, "right")
        ref = oracle.group_by_pairs(a[lo:hi], b[lo:hi], v[lo:hi])
        olo, ohi = np.searchsorted(got["a"], av, "left"), np.searchsorted(got["a"], av, "right")
        for col in ("a", "b", "count", "sum_i64", "min_i64", "max_i64"):
            assert np.array_equal(got[col][olo:ohi], ref[col]), (int(av), col)


@pytest.mark.timeout(900)
def test_batched_wave_full_size(ctx):
    # one wave of the batched configuration as the benchmark forms it: the
    # first instances of the 10,000-instance recipe (rows log-uniform 1e3..1e7,
    # distinct/rows log-uniform 1e-4..1, seed 6) up to 2e8 rows, in one call
    import torch
    import datagen
    import datagen.device as dgd
    rng = np.random.default_rng(6)
    count = 10_000
    rows = np.exp(rng.uniform(np.log(1e3), np.log(1e7), count)).round().astype(np.int64)
    ratio = np.exp(rng.uniform(np.log(1e-4), 0.0, count))
    d = np.maximum(1, np.round(rows * ratio)).astype(np.int64)
    cut = int(np.searchsorted(np.cumsum(rows), 200_000_000, "right"))
    say("case full-size batched wave: %d instances, %d rows" % (cut, int(rows[:cut].sum())))
    inputs = []
    for i in range(cut):
        seed = datagen.substream_seed(6, i)
        kk = dgd.keys(datagen.substream_seed(seed, 1), int(rows[i]), int(d[i]), 0.0)
        vv = dgd.uniform_i64(datagen.substream_seed(seed, 2), int(rows[i]))
        inputs.append((kk, vv, None))
    need = isa.lib().isa_batch_workspace_bytes(cut, (isa.isa_input * cut)(*[
        isa.isa_input(kk.data_ptr(), vv.data_ptr(), None, kk.numel()) for kk, vv, _ in inputs]), isa.ISA_INT_AGGS)
    res, status = isa.batch_run(ctx, inputs, aggs=isa.ISA_INT_AGGS, mem_budget=int(need))
    torch.cuda.synchronize()
    assert status == isa.ISA_OK
    t0 = time.time()
    for i in range(cut):
        k = to_np(inputs[i][0], np.uint64)
        v = to_np(inputs[i][1], np.int64)
        got = _host(res[i])
        assert (got["keys"][1:] > got["keys"][:-1]).all(), i
        ref = oracle.group_by(k, v, None, threads=min(ORACLE_THREADS, oracle.nproc()))
        for col in ("keys", "count", "sum_i64", "min_i64", "max_i64"):
            assert np.array_equal(got[col], ref[col]), (i, col)
    say("  oracle on every instance: %.1f s" % (time.time() - t0))

"""GPU parity of the sorted-input path (in-stream aggregation without a sort)
against the CPU oracle: the same grouping as for the unsorted input."""
import numpy as np
import pytest

import datagen
import paper_2010_00152_amd as isa
from tests.gpu_util import compare, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = isa.Context(0)
    yield c
    c.close()


def run_sorted(ctx, k, v, f, aggs=isa.ISA_ALL, capacity=None, check=True):
    res, status, g = isa.group_by_sorted(ctx, to_dev(k), to_dev(v), to_dev(f), aggs=aggs, capacity=capacity,
                                         check=check)
    out = {}
    for c, t in res.items():
        out[c] = to_np(t, {"keys": np.uint64, "count": np.uint64, "sum_f64": np.float64}.get(c, np.int64))
    return out, status, g


def sort_rows(k, v, f):
    o = np.argsort(k, kind="stable")
    return k[o], v[o], f[o]


@pytest.mark.parametrize("n,d", [(1, 1), (4095, 100), (4096, 4096), (4097, 3), (100_003, 20_000),
                                 (1_000_000, 300)])
def test_sorted_matches_oracle(ctx, n, d):
    say("case sorted n=%d d=%d" % (n, d))
    k, v, f = datagen.plain_input(31 + n % 7, n, d, 0.9, with_f64=True)
    k, v, f = sort_rows(k, v, f)
    got, status, g = run_sorted(ctx, k, v, f)
    compare(got, k, v, f, isa.ISA_ALL, "sorted %d" % n)


def test_sorted_long_groups_and_tile_edges(ctx):
    # groups far longer than a tile, groups ending exactly on tile edges,
    # single rows between long groups, and the largest key value
    say("case sorted long groups")
    sizes = [1, 4096, 4095, 1, 4097, 200_000, 3, 8192, 1, 1_000_000, 5, 4096 * 7, 2]
    keys = np.concatenate([np.full(s, i * 1000 + 7, np.uint64) for i, s in enumerate(sizes)] +
                          [np.full(9000, (1 << 64) - 1, np.uint64)])
    n = keys.shape[0]
    v = datagen.uniform_i64(33, n)
    f = datagen.normal_f64(34, n)
    got, status, g = run_sorted(ctx, keys, v, f)
    compare(got, keys, v, f, isa.ISA_ALL, "long groups")
    assert g == len(sizes) + 1


def test_sorted_one_key(ctx):
    say("case sorted one key")
    n = 3_000_001
    k = np.full(n, 42, np.uint64)
    v = datagen.uniform_i64(35, n)
    f = datagen.normal_f64(36, n)
    got, status, g = run_sorted(ctx, k, v, f)
    compare(got, k, v, f, isa.ISA_ALL, "one key")


def test_sorted_all_distinct_int_aggs(ctx):
    say("case sorted distinct")
    n = 777_777
    k = np.sort(datagen.key_of_rank(np.arange(n, dtype=np.uint64)))
    v = datagen.uniform_i64(37, n)
    got, status, g = run_sorted(ctx, k, v, None, aggs=isa.ISA_INT_AGGS)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "distinct")


def test_sorted_rejects_unsorted_and_truncates(ctx):
    say("case sorted errors")
    k = np.arange(10_000, dtype=np.uint64)
    k[5000], k[5001] = k[5001], k[5000]
    v = np.zeros(10_000, np.int64)
    with pytest.raises(isa.InsortError) as e:
        run_sorted(ctx, k, v, None, aggs=isa.ISA_INT_AGGS)
    assert e.value.status == isa.ISA_EINVAL
    k = np.repeat(np.arange(100, dtype=np.uint64), 50)
    v = np.zeros(5000, np.int64)
    got, status, g = run_sorted(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, capacity=99, check=False)
    assert status == isa.ISA_ETRUNC and g == 100

"""GPU parity of count(*) + count(distinct x) group by g (one sort on the
normalized pair key, then an in-stream regrouping on g) against the oracle."""
import numpy as np
import pytest

import oracle
import paper_2010_00152_amd as isa
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    c = isa.Context(0)
    yield c
    c.close()


def reference(g, x):
    # signed int32 order through the order-preserving map v ^ 2^31 to uint32
    gu = (g.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64)
    xu = (x.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64)
    r = oracle.count_distinct(gu, xu)
    keys = (r["keys"].astype(np.uint32) ^ np.uint32(0x80000000)).view(np.int32)
    return keys, r["count"], r["distinct"]


def run(ctx, g, x, **kw):
    res, status, n = isa.count_distinct(ctx, to_dev(g), to_dev(x), **kw)
    return to_np(res["g"], np.int32), to_np(res["count"], np.int64), to_np(res["distinct"], np.int64), status, n


@pytest.mark.parametrize("n,ng,nx,seed", [(1, 1, 1, 1), (5000, 7, 40, 2), (300_000, 1000, 5000, 3),
                                          (1_000_000, 50, 200_000, 4)])
def test_count_distinct_matches_oracle(ctx, n, ng, nx, seed):
    say("case count distinct n=%d" % n)
    rng = np.random.default_rng(seed)
    gv = rng.integers(-2**31, 2**31, ng, dtype=np.int64).astype(np.int32)
    xv = rng.integers(-2**31, 2**31, nx, dtype=np.int64).astype(np.int32)
    g = gv[rng.integers(0, ng, n)]
    x = xv[rng.integers(0, nx, n)]
    kg, kc, kd = reference(g, x)
    og, oc, od, status, m = run(ctx, g, x)
    assert status == isa.ISA_OK and m == kg.shape[0]
    assert np.array_equal(og, kg)
    assert np.array_equal(oc.astype(np.uint64), kc)
    assert np.array_equal(od.astype(np.uint64), kd)


def test_count_distinct_spilling_and_brute_force(ctx):
    # a budget far below the distinct pairs: the pair grouping spills runs and
    # wide-merges them; checked against a dictionary as well as the oracle
    say("case count distinct spilling")
    rng = np.random.default_rng(9)
    n = 2_000_000
    g = rng.integers(-300, 300, n).astype(np.int32)
    x = rng.integers(0, 4000, n).astype(np.int32)
    og, oc, od, status, m = run(ctx, g, x, mem_budget=16 << 20)
    kg, kc, kd = reference(g, x)
    assert np.array_equal(og, kg) and np.array_equal(oc.astype(np.uint64), kc)
    assert np.array_equal(od.astype(np.uint64), kd)
    pairs = np.unique((g.astype(np.int64) << 32) | (x.astype(np.int64) & 0xFFFFFFFF))
    ug, cnt = np.unique(g, return_counts=True)
    assert np.array_equal(og, ug) and np.array_equal(oc, cnt)
    assert np.array_equal(od, np.bincount(np.searchsorted(ug, (pairs >> 32).astype(np.int32)), minlength=ug.size))


def test_count_distinct_errors(ctx):
    say("case count distinct errors")
    import torch
    g = np.arange(1000, dtype=np.int32) % 10
    x = np.arange(1000, dtype=np.int32)
    og, oc, od, status, m = run(ctx, g, x, capacity=5, check=False)
    assert status == isa.ISA_ETRUNC and m == 10
    small = torch.empty(8 * 1000 + 16 * 10, dtype=torch.uint8, device="cuda")  # room for 10 pairs only
    with pytest.raises(isa.InsortError) as e:
        isa.count_distinct(ctx, to_dev(g), to_dev(x), scratch=small)
    assert e.value.status == isa.ISA_EBUDGET

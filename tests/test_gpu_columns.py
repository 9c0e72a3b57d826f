"""GPU parity of grouping on multi-column keys with offset-value codes
(isa_group_by_columns) against the offset-value-code oracle (oracle/ovc.py):
group keys, counts and int64 sums bit-exact against ovc.group_rows, min and
max against numpy over the oracle's sorted order, duplicate removal against
ovc.distinct_rows, every code of the sorted stream against ovc.stream_codes,
and the column values compared against the count the codes imply (at most
N x K, Section 5)."""
import numpy as np
import pytest

import paper_2010_00152_amd as isa
from oracle import ovc
from tests.gpu_util import say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = isa.Context(0)
    yield c
    c.close()


def _run(ctx, rows, v, aggs, codes=False, capacity=None, check=True):
    import torch
    cols = [to_dev(np.ascontiguousarray(rows[:, c])) for c in range(rows.shape[1])]
    vd = to_dev(v) if v is not None else None
    res, cd, cmp, st, g = isa.group_by_columns(ctx, cols, vd, aggs=aggs, codes=codes, capacity=capacity,
                                               check=check)
    torch.cuda.synchronize()
    out = {c: to_np(t, np.uint64 if c == "count" else np.int64) for c, t in res.items() if c != "cols"}
    keys = np.stack([to_np(t, np.int64) for t in res["cols"]], axis=1) if res["cols"] else None
    cdh = {k: to_np(t, np.int64 if k == "value" else np.int32) for k, t in cd.items()} if cd else None
    return keys, out, cdh, cmp, st, g


def _ref_min_max(rows, v):
    order = np.lexsort(rows.T[::-1])
    srt, val = rows[order], v[order]
    heads = np.flatnonzero(np.r_[True, (srt[1:] != srt[:-1]).any(axis=1)])
    return np.minimum.reduceat(val, heads), np.maximum.reduceat(val, heads)


@pytest.mark.parametrize("n,K,domain,seed", [(1, 3, 100, 1), (4095, 3, 100, 2), (4097, 4, 10, 3),
                                             (200_000, 3, 100, 4), (65_537, 2, 7, 5), (300_000, 5, 4, 6)])
def test_columns_match_the_ovc_oracle(ctx, n, K, domain, seed):
    say("case columns n=%d K=%d domain=%d" % (n, K, domain))
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, domain, size=(n, K)).astype(np.int64)
    v = rng.integers(-1_000_000, 1_000_000, n).astype(np.int64)
    aggs = isa.ISA_COUNT | isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64
    keys, out, cd, cmp, st, g = _run(ctx, rows, v, aggs, codes=True)
    assert st == isa.ISA_OK
    rk, rc, rs = ovc.group_rows(rows, v, domain)
    assert g == rk.shape[0]
    assert np.array_equal(keys, rk)
    assert np.array_equal(out["count"], rc.astype(np.uint64))
    assert np.array_equal(out["sum_i64"], rs)
    mn, mx = _ref_min_max(rows, v)
    assert np.array_equal(out["min_i64"], mn) and np.array_equal(out["max_i64"], mx)
    # the codes of the sorted stream, in the oracle's ascending form
    srt = rows[np.lexsort(rows.T[::-1])]
    _, asc = ovc.stream_codes(srt, domain)
    off = cd["offset"].astype(np.int64)
    got_asc = np.where(off < K, (K - off) * domain + cd["value"], 0)
    assert np.array_equal(got_asc, asc)
    # column values compared: offset + 1 for a row that differs, K for a duplicate
    ref_off = np.where(asc != 0, K - asc // domain, K)
    expect = int(np.minimum(ref_off[1:] + 1, K).sum())
    assert cmp == expect and cmp <= (n - 1) * K


def test_duplicate_removal_and_count_only(ctx):
    say("case columns duplicate removal")
    rng = np.random.default_rng(11)
    rows = rng.integers(0, 9, size=(120_000, 3)).astype(np.int64)
    keys, out, _, _, st, g = _run(ctx, rows, None, 0)
    uk, uc = ovc.distinct_rows(rows, 9)
    assert st == isa.ISA_OK and np.array_equal(keys, uk) and out == {}
    keys, out, _, _, st, g = _run(ctx, rows, None, isa.ISA_COUNT)
    assert np.array_equal(keys, uk) and np.array_equal(out["count"], uc.astype(np.uint64))


def test_signed_extremes_against_brute_force(ctx):
    # any int64 values, signed order per column, with constant columns (no
    # radix pass) and duplicates; a dictionary over row tuples is the oracle
    say("case columns signed extremes")
    rng = np.random.default_rng(12)
    n = 20_000
    pool = np.array([np.iinfo(np.int64).min, -5, -1, 0, 1, 7, np.iinfo(np.int64).max], np.int64)
    rows = np.stack([pool[rng.integers(0, 7, n)], np.full(n, 42, np.int64),
                     rng.integers(-3, 3, n).astype(np.int64) * (1 << 40)], axis=1)
    v = rng.integers(-10, 10, n).astype(np.int64)
    aggs = isa.ISA_COUNT | isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64
    keys, out, _, _, st, g = _run(ctx, rows, v, aggs)
    d = {}
    for r, x in zip(map(tuple, rows.tolist()), v.tolist()):
        c, s_, lo, hi = d.get(r, (0, 0, x, x))
        d[r] = (c + 1, s_ + x, min(lo, x), max(hi, x))
    ks = sorted(d)
    assert g == len(ks)
    assert [tuple(r) for r in keys.tolist()] == ks
    assert out["count"].tolist() == [d[k][0] for k in ks]
    assert out["sum_i64"].tolist() == [d[k][1] for k in ks]
    assert out["min_i64"].tolist() == [d[k][2] for k in ks]
    assert out["max_i64"].tolist() == [d[k][3] for k in ks]
    # every column constant: one group
    same = np.zeros((5000, 2), np.int64)
    keys, out, _, cmp, st, g = _run(ctx, same, None, isa.ISA_COUNT)
    assert g == 1 and out["count"].tolist() == [5000] and cmp == 4999 * 2


def test_columns_truncation_and_errors(ctx):
    say("case columns truncation")
    rng = np.random.default_rng(13)
    rows = rng.integers(0, 50, size=(30_000, 2)).astype(np.int64)
    rk, rc, _ = ovc.group_rows(rows, np.zeros(30_000, np.int64), 50)
    G = rk.shape[0]
    keys, out, _, _, st, g = _run(ctx, rows, None, isa.ISA_COUNT, capacity=G - 3, check=False)
    assert st == isa.ISA_ETRUNC and g == G
    with pytest.raises(isa.InsortError) as e:
        _run(ctx, rows, None, isa.ISA_SUM_I64)       # sum without a value column
    assert e.value.status == isa.ISA_EINVAL

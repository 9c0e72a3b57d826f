"""Pins for the CPU oracle: it is checked against things other than itself --
brute-force hashing, Python's correctly rounded math.fsum, numpy sort and
reductions on special cases, closed-form invariants, and hand-computed cases.
"""
import math
from collections import defaultdict

import numpy as np
import pytest

import datagen
import oracle

U64 = 1 << 64


def brute_force(keys, v=None, f=None):
    """Dictionary-based grouping: an independent definition of the result."""
    groups = defaultdict(list)
    for i, k in enumerate(keys.tolist()):
        groups[k].append(i)
    out = {"keys": [], "count": [], "sum_i64": [], "min_i64": [], "max_i64": [], "sum_f64": []}
    for k in sorted(groups):
        rows = groups[k]
        out["keys"].append(k)
        out["count"].append(len(rows))
        if v is not None:
            vals = [int(v[r]) for r in rows]
            s = sum(vals) % U64
            if s >= 1 << 63:
                s -= U64
            out["sum_i64"].append(s)
            out["min_i64"].append(min(vals))
            out["max_i64"].append(max(vals))
        if f is not None:
            out["sum_f64"].append(math.fsum(float(f[r]) for r in rows))
    return out


def assert_same(got, want, with_v=True, with_f=False):
    assert got["keys"].tolist() == want["keys"]
    assert got["count"].tolist() == want["count"]
    if with_v:
        assert got["sum_i64"].tolist() == want["sum_i64"]
        assert got["min_i64"].tolist() == want["min_i64"]
        assert got["max_i64"].tolist() == want["max_i64"]
    if with_f:
        # math.fsum is correctly rounded, and so is the oracle: bit-equal
        assert got["sum_f64"].tobytes() == np.array(want["sum_f64"], np.float64).tobytes()


@pytest.mark.parametrize("seed,n,d,s", [(1, 1, 1, 0), (2, 2, 1, 0), (3, 10, 3, 0),
                                        (4, 100, 7, 0.8), (5, 1000, 50, 1.2),
                                        (6, 3000, 3000, 0), (7, 5000, 200, 0.5)])
def test_oracle_matches_brute_force(seed, n, d, s):
    k, v, f = datagen.plain_input(seed, n, d, s, with_f64=True)
    got = oracle.group_by(k, v, f)
    assert_same(got, brute_force(k, v, f), with_f=True)


def test_empty_input():
    got = oracle.group_by(np.empty(0, np.uint64), np.empty(0, np.int64), np.empty(0))
    assert got["keys"].shape == (0,)


def test_single_row():
    got = oracle.group_by(np.array([7], np.uint64), np.array([-3]), np.array([2.5]))
    assert got["keys"].tolist() == [7]
    assert got["count"].tolist() == [1]
    assert got["sum_i64"].tolist() == [-3]
    assert got["min_i64"].tolist() == [-3] and got["max_i64"].tolist() == [-3]
    assert got["sum_f64"].tolist() == [2.5]


def test_unsigned_key_order():
    # keys compare as unsigned: 2^63 and 2^64-1 sort after small keys
    k = np.array([U64 - 1, 0, 1 << 63, 5, (1 << 63) - 1, 0], np.uint64)
    got = oracle.group_by(k, np.arange(6, dtype=np.int64))
    assert got["keys"].tolist() == [0, 5, (1 << 63) - 1, 1 << 63, U64 - 1]
    assert got["count"].tolist() == [2, 1, 1, 1, 1]
    assert got["sum_i64"].tolist() == [1 + 5, 3, 4, 2, 0]


def test_int64_sum_wraps_and_extremes():
    big = np.iinfo(np.int64).max
    small = np.iinfo(np.int64).min
    k = np.array([1, 1, 1, 2, 2], np.uint64)
    v = np.array([big, big, 5, small, small], np.int64)
    got = oracle.group_by(k, v)
    # (2*(2^63-1) + 5) mod 2^64 as int64 = 3 ; 2*(-2^63) mod 2^64 = 0
    assert got["sum_i64"].tolist() == [3, 0]
    assert got["min_i64"].tolist() == [5, small]
    assert got["max_i64"].tolist() == [big, small]


def test_all_distinct_is_sorted_input():
    # O = I: the result is the input sorted on the key, count 1, sum=min=max=v
    k, v, f = datagen.plain_input(11, 20000, 1 << 40, 0.0, with_f64=True)
    assert np.unique(k).shape[0] == k.shape[0]
    got = oracle.group_by(k, v, f)
    order = np.argsort(k, kind="stable")
    assert np.array_equal(got["keys"], k[order])
    assert np.all(got["count"] == 1)
    assert np.array_equal(got["sum_i64"], v[order])
    assert np.array_equal(got["min_i64"], v[order])
    assert np.array_equal(got["max_i64"], v[order])
    assert np.array_equal(got["sum_f64"], f[order])


def test_single_key_is_plain_reduction():
    # O = 1: count/sum/min/max are numpy's reductions over the whole column
    n = 50000
    k = np.full(n, 0xDEADBEEF, np.uint64)
    v = datagen.uniform_i64(3, n)
    f = datagen.normal_f64(4, n)
    got = oracle.group_by(k, v, f)
    assert got["keys"].tolist() == [0xDEADBEEF]
    assert got["count"].tolist() == [n]
    assert got["sum_i64"].tolist() == [int(v.sum())]
    assert got["min_i64"].tolist() == [int(v.min())]
    assert got["max_i64"].tolist() == [int(v.max())]
    assert got["sum_f64"][0] == math.fsum(f.tolist())


def test_sorted_input_matches_run_boundaries():
    # already-sorted input: groups are the maximal runs of equal keys
    k = np.sort(datagen.plain_input(12, 30000, 700, 0.9)[0])
    v = datagen.uniform_i64(13, k.shape[0])
    got = oracle.group_by(k, v)
    starts = np.flatnonzero(np.r_[True, k[1:] != k[:-1]])
    ends = np.r_[starts[1:], k.shape[0]]
    assert np.array_equal(got["keys"], k[starts])
    assert np.array_equal(got["count"], (ends - starts).astype(np.uint64))
    assert np.array_equal(got["sum_i64"], np.add.reduceat(v, starts))
    assert np.array_equal(got["min_i64"], np.minimum.reduceat(v, starts))
    assert np.array_equal(got["max_i64"], np.maximum.reduceat(v, starts))


@pytest.mark.parametrize("seed,s", [(21, 0.0), (22, 0.8), (23, 1.2)])
def test_invariants(seed, s):
    n = 200_000
    k, v, f = datagen.plain_input(seed, n, 50_000, s, with_f64=True)
    got = oracle.group_by(k, v, f)
    assert np.all(got["keys"][1:] > got["keys"][:-1])               # I1
    assert int(got["count"].sum()) == n                              # I2
    assert int(got["sum_i64"].sum()) == int(v.sum())                 # I3
    assert int(got["min_i64"].min()) == int(v.min())                 # I4
    assert int(got["max_i64"].max()) == int(v.max())
    assert np.array_equal(got["keys"], np.unique(k))
    assert math.isclose(math.fsum(got["sum_f64"].tolist()), math.fsum(f.tolist()),
                        rel_tol=0, abs_tol=1e-9)


def test_permutation_invariance():
    k, v, f = datagen.plain_input(31, 40000, 3000, 1.0, with_f64=True)
    p = np.random.default_rng(0).permutation(k.shape[0])
    a = oracle.group_by(k, v, f)
    b = oracle.group_by(k[p], v[p], f[p])
    for c in a:
        assert a[c].tobytes() == b[c].tobytes()


@pytest.mark.parametrize("case", ["cancel", "tiny", "huge", "mixed", "ties"])
def test_exact_sum_matches_fsum(case):
    rng = np.random.default_rng(hash(case) % 1000)
    if case == "cancel":
        x = np.array([1e100, 1.0, -1e100, 1e-100, -1.0, 3.0])
    elif case == "tiny":
        x = np.array([5e-324, 5e-324, -1e-310, 2.2e-308, 1e-320] * 7)
    elif case == "huge":
        x = np.array([1.7e308, -1.7e308, 1.6e308, 1e292, -1e292, 1.0])
    elif case == "mixed":
        x = rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000)
    else:  # exact halfway cases that need correct tie-breaking
        x = np.array([1.0, 2.0 ** -53, 2.0 ** -106, 1.0, 2.0 ** -53])
    assert oracle.exact_sum(x) == math.fsum(x.tolist())


def test_exact_sum_nonfinite():
    assert math.isnan(oracle.exact_sum(np.array([1.0, np.inf, -np.inf])))
    assert oracle.exact_sum(np.array([1.0, np.inf, 2.0])) == np.inf
    assert math.isnan(oracle.exact_sum(np.array([np.nan, 1.0])))
    assert oracle.exact_sum(np.array([])) == 0.0


def test_pairs_match_brute_force():
    a, b, v = datagen.segmented_input(5, 20000, n_a=20, b_per_a=300)
    got = oracle.group_by_pairs(a, b, v)
    groups = defaultdict(list)
    for i in range(a.shape[0]):
        groups[(int(a[i]), int(b[i]))].append(int(v[i]))
    keys = sorted(groups)   # Python tuple order on signed ints
    assert list(zip(got["a"].tolist(), got["b"].tolist())) == keys
    assert got["count"].tolist() == [len(groups[kk]) for kk in keys]
    assert got["sum_i64"].tolist() == [sum(groups[kk]) for kk in keys]
    assert got["min_i64"].tolist() == [min(groups[kk]) for kk in keys]
    assert got["max_i64"].tolist() == [max(groups[kk]) for kk in keys]


def test_pairs_signed_order():
    a = np.array([-1, 1, -1, 0, -2147483648, 2147483647], np.int32)
    b = np.array([5, -5, -7, 0, 1, -1], np.int32)
    got = oracle.group_by_pairs(a, b, np.zeros(6, np.int64))
    assert list(zip(got["a"].tolist(), got["b"].tolist())) == \
        [(-2147483648, 1), (-1, -7), (-1, 5), (0, 0), (1, -5), (2147483647, -1)]


def test_count_distinct_brute_force():
    n = 20000
    g = datagen.uniform_ranks(41, n, 50)
    x = datagen.uniform_ranks(42, n, 300)
    got = oracle.count_distinct(g, x)
    rows = defaultdict(list)
    for gi, xi in zip(g.tolist(), x.tolist()):
        rows[gi].append(xi)
    ks = sorted(rows)
    assert got["keys"].tolist() == ks
    assert got["count"].tolist() == [len(rows[kk]) for kk in ks]
    assert got["distinct"].tolist() == [len(set(rows[kk])) for kk in ks]


@pytest.mark.parametrize("threads", [2, 3, 8, 0])
@pytest.mark.parametrize("seed,n,d,s", [(11, 1, 1, 0), (12, 5, 5, 0), (13, 1000, 1, 0),
                                        (14, 20000, 300, 1.2), (15, 200000, 50000, 0.8),
                                        (16, 100000, 100000, 0)])
def test_threaded_oracle_equals_single_thread(threads, seed, n, d, s):
    # the key-range split over threads gives the single-threaded result, bit for bit
    k, v, f = datagen.plain_input(seed, n, d, s, with_f64=True)
    one = oracle.group_by(k, v, f)
    many = oracle.group_by(k, v, f, threads=threads)
    for col in one:
        assert one[col].tobytes() == many[col].tobytes(), col


def test_threaded_oracle_brute_force_and_extreme_keys():
    rng = np.random.default_rng(17)
    k = rng.choice(np.array([0, 1, 2, 1 << 63, (1 << 64) - 2, (1 << 64) - 1], np.uint64), 3000)
    v = rng.integers(-(1 << 62), 1 << 62, 3000, dtype=np.int64)
    f = rng.standard_normal(3000)
    f[5] = np.inf
    got = oracle.group_by(k, v, f, threads=4)
    want = brute_force(k, v, f)
    assert got["keys"].tolist() == want["keys"]
    assert got["count"].tolist() == want["count"]
    assert got["sum_i64"].tolist() == want["sum_i64"]
    assert got["min_i64"].tolist() == want["min_i64"]
    assert got["max_i64"].tolist() == want["max_i64"]
    # finite groups: correctly rounded; the group holding +inf sums to +inf
    fin = np.isfinite(np.array(want["sum_f64"]))
    assert np.array_equal(got["sum_f64"][fin], np.array(want["sum_f64"])[fin])
    assert np.isinf(got["sum_f64"][~fin]).all()


def test_threaded_oracle_without_value_columns():
    k, _, _ = datagen.plain_input(18, 50000, 700, 0.5, with_f64=False)
    one = oracle.group_by(k)
    many = oracle.group_by(k, threads=5)
    assert set(one) == set(many) == {"keys", "count"}
    for col in one:
        assert np.array_equal(one[col], many[col])

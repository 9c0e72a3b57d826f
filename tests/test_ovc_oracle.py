"""Pins for the offset-value-code oracle: the paper's worked table, the
ordering property of codes against a common base (brute force over a small
domain), the property that lets a merge keep a loser's code, and duplicate
removal against numpy's unique rows."""
import itertools
import os

import numpy as np
import pytest

from oracle import ovc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ovc_table.txt")


def _golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(x) for x in line.split()])
    return np.array(rows, dtype=np.int64)


def test_paper_table():
    g = _golden()
    rows, offs, desc, asc = g[:, :4], g[:, 4], g[:, 5], g[:, 6]
    d, a = ovc.stream_codes(rows, domain=100)
    assert np.array_equal(d, desc)
    assert np.array_equal(a, asc)
    got_offs = [0] + [ovc.offset_of(rows[i], rows[i - 1]) for i in range(1, len(rows))]
    assert got_offs == list(offs)


def _lex_gt(x, y):
    return tuple(x) > tuple(y)


# all rows of 3 columns over values 0..3
DOMAIN, K = 4, 3
ALL = [tuple(r) for r in itertools.product(range(DOMAIN), repeat=K)]


def test_codes_order_rows_coded_against_one_base():
    # for x, y >= base: a larger ascending code (a smaller descending code)
    # means a larger row; equal codes leave the rows undecided only when they
    # agree up to and including the column the codes describe
    for b in ALL:
        above = [r for r in ALL if r >= b]
        codes = {r: ovc.code_pair(r, b, DOMAIN) for r in above}
        for x in above:
            dx, ax = codes[x]
            for y in above:
                dy, ay = codes[y]
                if ax > ay:
                    assert _lex_gt(x, y), (b, x, y)
                if dx < dy:
                    assert _lex_gt(x, y), (b, x, y)
                assert (ax == ay) == (dx == dy)
                if ax == ay:
                    off = ovc.offset_of(x, b)
                    assert off == ovc.offset_of(y, b)
                    assert x[:off + 1] == y[:off + 1]


def test_loser_keeps_its_code():
    # two rows coded against one base: the smaller one (the winner of an
    # ascending merge) has the smaller ascending code, and the larger one's
    # code against the winner equals its code against the base
    for b in ALL:
        above = [r for r in ALL if r >= b]
        for x in above:
            ax = ovc.code_pair(x, b, DOMAIN)[1]
            for y in above:
                ay = ovc.code_pair(y, b, DOMAIN)[1]
                if ay < ax:
                    assert ovc.code_pair(x, y, DOMAIN)[1] == ax, (b, x, y)


def test_first_row_and_duplicates():
    d, a = ovc.stream_codes([(0, 0, 0), (0, 0, 0), (0, 0, 1)], domain=DOMAIN)
    assert list(a) == [K * DOMAIN + 0, 0, 1 * DOMAIN + 1]
    assert list(d) == [DOMAIN, K * DOMAIN, 2 * DOMAIN + DOMAIN - 1]


@pytest.mark.parametrize("n,k,dom,seed", [(0, 3, 5, 0), (1, 2, 3, 1), (500, 3, 4, 2), (2000, 5, 3, 3),
                                          (3000, 2, 100, 4)])
def test_distinct_rows_match_numpy(n, k, dom, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, dom, size=(n, k), dtype=np.int64)
    u, c = ovc.distinct_rows(rows, dom)
    if n == 0:
        assert u.shape[0] == 0 and c.shape[0] == 0
        return
    ref_u, ref_c = np.unique(rows, axis=0, return_counts=True)
    assert np.array_equal(u, ref_u)
    assert np.array_equal(c, ref_c)
    assert c.sum() == n


@pytest.mark.parametrize("n,k,dom,seed", [(1, 3, 4, 5), (800, 3, 4, 6), (2000, 4, 3, 7)])
def test_group_rows_match_brute_force(n, k, dom, seed):
    rng = np.random.default_rng(seed)
    rows = rng.integers(0, dom, size=(n, k), dtype=np.int64)
    vals = rng.integers(-(1 << 62), 1 << 62, size=n, dtype=np.int64)
    keys, cnt, sums = ovc.group_rows(rows, vals, dom)
    ref = {}
    for r, v in zip(map(tuple, rows.tolist()), vals.tolist()):
        c, s = ref.get(r, (0, 0))
        ref[r] = (c + 1, (s + v + (1 << 63)) % (1 << 64) - (1 << 63))
    want = sorted(ref)
    assert [tuple(x) for x in keys.tolist()] == want
    assert cnt.tolist() == [ref[r][0] for r in want]
    assert sums.tolist() == [ref[r][1] for r in want]


def _runs(rng, n_runs, k, dom, max_len):
    return [sorted(map(tuple, rng.integers(0, dom, size=(int(rng.integers(0, max_len + 1)), k)).tolist()))
            for _ in range(n_runs)]


@pytest.mark.parametrize("n_runs,k,dom,seed", [(1, 3, 3, 0), (2, 4, 2, 1), (3, 2, 5, 2), (5, 4, 3, 3),
                                               (8, 3, 4, 4), (13, 5, 2, 5), (6, 1, 7, 6)])
def test_tree_of_losers_merge_with_codes(n_runs, k, dom, seed):
    # the merge outputs every row in order, the codes it carries out are the
    # output stream's own codes, and it compares at most N x K column values
    # (Section 5: offset-value codes bound column comparisons by rows times
    # columns)
    rng = np.random.default_rng(seed)
    for _ in range(20):
        runs = _runs(rng, n_runs, k, dom, 40)
        out, codes, cmp = ovc.merge_runs(runs, dom)
        rows = sorted(r for run in runs for r in run)
        assert out == rows
        if rows:
            assert list(codes) == list(ovc.stream_codes(out, dom)[1])
        assert cmp <= len(rows) * k


def test_merge_with_unique_leading_column_reads_no_other_column():
    # Section 5's first extreme case: when the first column is unique, codes
    # decide every comparison and no further column is compared
    rng = np.random.default_rng(9)
    lead = rng.permutation(600)
    rows = [(int(a),) + tuple(int(x) for x in rng.integers(0, 5, 3)) for a in lead]
    runs = [sorted(rows[i::7]) for i in range(7)]
    out, codes, cmp = ovc.merge_runs(runs, 600)
    assert out == sorted(rows)
    assert cmp == 0

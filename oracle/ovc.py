"""Offset-value codes of a sorted stream of multi-column rows.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Offset-value coding (Section 2, the discussion of efficient sorting and its
table of offset-value codes; Section 5 on column accesses) describes a row by
its position relative to an earlier row of the same sort order: the offset is
the number of leading key columns the row shares with that base row, and the
value is the row's own value in the first column where the two differ.  Both
are folded into one integer so that a single integer comparison orders two
rows coded against the same base.

For rows in ascending order on all K columns, each column value in
[0, domain):

* descending code = offset * domain + (domain - value)
* ascending code  = (K - offset) * domain + value

A row equal to its base has offset K: its descending code is K * domain and
its ascending code 0.  The first row of a stream is coded against a base that
differs from it in column 0 (offset 0).  The worked example of the paper's
table takes domain = 100 and K = 4.

This module holds no arithmetic of the GPU path; the GPU path has no
multi-column keys.
"""
from __future__ import annotations

import numpy as np


def offset_of(row, base) -> int:
    """Number of leading columns in which row equals base."""
    k = 0
    for a, b in zip(row, base):
        if a != b:
            break
        k += 1
    return k


def code_pair(row, base, domain: int):
    """(descending, ascending) code of row relative to base (row >= base in
    ascending order; base None: the first row of a stream)."""
    K = len(row)
    off = 0 if base is None else offset_of(row, base)
    if off == K:
        return K * domain, 0
    v = int(row[off])
    return off * domain + (domain - v), (K - off) * domain + v


def stream_codes(rows, domain: int):
    """Descending and ascending codes of every row of a sorted stream, each
    relative to its predecessor (the first row: offset 0)."""
    rows = [tuple(int(x) for x in r) for r in rows]
    desc, asc = [], []
    prev = None
    for r in rows:
        d, a = code_pair(r, prev, domain)
        desc.append(d)
        asc.append(a)
        prev = r
    return np.array(desc, dtype=np.int64), np.array(asc, dtype=np.int64)


def distinct_rows(rows, domain: int):
    """Sort-based duplicate removal with ascending codes: sort the rows, code
    each against its predecessor, keep the rows whose code is nonzero, and
    count each kept row's duplicates.  Returns (unique rows, counts)."""
    rows = np.asarray(rows, dtype=np.int64)
    if rows.shape[0] == 0:
        return rows.reshape(0, rows.shape[1] if rows.ndim == 2 else 0), np.zeros(0, np.int64)
    order = np.lexsort(rows.T[::-1])
    srt = rows[order]
    _, asc = stream_codes(srt, domain)
    heads = np.flatnonzero(asc != 0)
    counts = np.diff(np.append(heads, srt.shape[0]))
    return srt[heads], counts


def group_rows(rows, values, domain: int):
    """Grouping on a multi-column key with count(*) and sum of an int64 value:
    sort on all key columns, then one in-stream pass in which a nonzero
    ascending code against the predecessor starts a group (in-stream grouping
    of sorted input, Section 2.1, decided by offset-value codes).  Returns
    (group keys, counts, sums); sums wrap modulo 2^64 like int64 addition."""
    rows = np.asarray(rows, dtype=np.int64)
    values = np.asarray(values, dtype=np.int64)
    if rows.shape[0] == 0:
        return rows, np.zeros(0, np.int64), np.zeros(0, np.int64)
    order = np.lexsort(rows.T[::-1])
    srt, val = rows[order], values[order]
    _, asc = stream_codes(srt, domain)
    heads = np.flatnonzero(asc != 0)
    counts = np.diff(np.append(heads, srt.shape[0]))
    with np.errstate(over="ignore"):
        sums = np.add.reduceat(val, heads)
    return srt[heads], counts, sums


def merge_runs(runs, domain: int):
    """Merge sorted runs of K-column rows with a tree-of-losers priority queue
    whose comparisons use offset-value codes (Section 2: tree-of-losers
    priority queues and offset-value coding; Section 5: column accesses).

    Every row enters with its ascending code against its run predecessor (a
    run's first row against a base below every row: offset 0).  All codes
    compared at a node are relative to the same row, the last one output, so
    unequal codes decide a comparison alone; equal codes continue with the
    columns after their offset, and the loser's code is recomputed from the
    first differing column.  Returns (output rows, their codes against their
    output predecessors, column comparisons made)."""
    runs = [[tuple(int(x) for x in r) for r in run] for run in runs]
    runs = [r for r in runs if r]
    if not runs:
        return [], [], 0
    K = len(runs[0][0])
    INF = None  # an exhausted input: loses to every row
    k = 1
    while k < len(runs):
        k *= 2
    pos = [0] * k
    cur = [None] * k
    code = [INF] * k
    for i, run in enumerate(runs):
        cur[i] = run[0]
        code[i] = K * domain + run[0][0] if K else 0
    comparisons = 0

    def play(a, b):
        """Winner and loser of inputs a, b (codes against one base); updates
        the loser's code against the winner."""
        nonlocal comparisons
        ca, cb = code[a], code[b]
        if ca is INF:
            return b, a
        if cb is INF:
            return a, b
        if ca != cb:
            return (a, b) if ca < cb else (b, a)
        off = K - ca // domain if ca else K
        for c in range(off + 1, K):
            comparisons += 1
            if cur[a][c] != cur[b][c]:
                w, l = (a, b) if cur[a][c] < cur[b][c] else (b, a)
                code[l] = (K - c) * domain + cur[l][c]
                return w, l
        w, l = (a, b) if a < b else (b, a)
        code[l] = 0
        return w, l

    # tree[1..k-1]: losers at internal nodes; leaves k..2k-1 are the inputs
    tree = [0] * k
    win = [0] * (2 * k)
    for i in range(k):
        win[k + i] = i
    for n in range(k - 1, 0, -1):
        w, l = play(win[2 * n], win[2 * n + 1])
        win[n], tree[n] = w, l
    champion = win[1] if k > 1 else 0
    out, out_codes = [], []
    while code[champion] is not INF:
        w = champion
        out.append(cur[w])
        out_codes.append(code[w])
        run = runs[w]
        pos[w] += 1
        if pos[w] < len(run):
            prev, row = run[pos[w] - 1], run[pos[w]]
            cur[w] = row
            code[w] = code_pair(row, prev, domain)[1]
        else:
            cur[w], code[w] = None, INF
        # replay from the leaf to the root against the stored losers
        cand = w
        n = (k + w) // 2
        while n >= 1:
            wn, ln = play(cand, tree[n])
            tree[n] = ln
            cand = wn
            n //= 2
        champion = cand
    return out, out_codes, comparisons

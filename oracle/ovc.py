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

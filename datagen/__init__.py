"""Seeded synthetic input generators, shared by the tests, the benchmark and
the oracle.  They hold none of the grouping method's arithmetic: they only
produce key and value columns.

All integer streams are counter-based SplitMix64 (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): element i of
the stream with seed s is ``mix(s + (i + 1) * GAMMA)``, where ``mix`` is the
published SplitMix64 finaliser.  Being counter-based, any sub-range can be
generated independently and identically on host or device.

Workload shapes (paper Section 3, Example 1 and Section 6; the synthetic
recipes stand in for the TPC-H and production inputs the paper mentions):

* key domain: ``d`` distinct uint64 values, value of rank r is ``mix(r ^ salt)``
  (a bijection, so the d values are distinct and unordered w.r.t. popularity);
* rank distribution: uniform over [0, d) or Zipf with exponent s over ranks
  1..d (P(r) proportional to r^-s) sampled by inversion of a uint64 CDF table;
* int64 value uniform in [-1e6, 1e6];
* float64 value standard normal (numpy PCG64 with the given seed).
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
KEY_SALT = np.uint64(0x5DEECE66D1234567)


def mix64(z):
    """SplitMix64 finaliser (a bijection on uint64)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream(seed: int, start: int, count: int):
    """Elements [start, start+count) of the SplitMix64 stream of ``seed``."""
    i = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * GAMMA
    return mix64(z)


def substream_seed(master: int, ident: int) -> int:
    """Per-instance seed derived from a master seed and an instance id."""
    v = (np.uint64(master & 0xFFFFFFFF) << np.uint64(32)) | np.uint64(ident & 0xFFFFFFFF)
    return int(mix64(np.array([v], dtype=np.uint64))[0])


def mulhi(x, m: int):
    """floor(x * m / 2^64) for uint64 x and 0 < m < 2^32 (exact)."""
    x = np.asarray(x, dtype=np.uint64)
    m = np.uint64(m)
    lo = x & np.uint64(0xFFFFFFFF)
    hi = x >> np.uint64(32)
    with np.errstate(over="ignore"):
        # x*m = hi*m*2^32 + lo*m ; both products < 2^64 since m < 2^32
        t = (lo * m) >> np.uint64(32)
        return (hi * m + t) >> np.uint64(32)


def mulhi64(x, m: int):
    """floor(x * m / 2^64) for uint64 x and any uint64 m (exact)."""
    x = np.asarray(x, dtype=np.uint64)
    mm = np.uint64(m)
    x_lo = x & np.uint64(0xFFFFFFFF)
    x_hi = x >> np.uint64(32)
    m_lo = mm & np.uint64(0xFFFFFFFF)
    m_hi = mm >> np.uint64(32)
    with np.errstate(over="ignore"):
        ll = x_lo * m_lo
        lh = x_lo * m_hi
        hl = x_hi * m_lo
        hh = x_hi * m_hi
        mid = (ll >> np.uint64(32)) + (lh & np.uint64(0xFFFFFFFF)) + (hl & np.uint64(0xFFFFFFFF))
        return hh + (lh >> np.uint64(32)) + (hl >> np.uint64(32)) + (mid >> np.uint64(32))


def key_of_rank(rank, salt: int = int(KEY_SALT)):
    """Domain value of a rank: a bijective mix, distinct for distinct ranks."""
    r = np.asarray(rank, dtype=np.uint64)
    return mix64(r ^ np.uint64(salt))


def uniform_ranks(seed: int, n: int, d: int, start: int = 0):
    """n ranks uniform over [0, d)."""
    return mulhi64(stream(seed, start, n), d)


def zipf_cdf_table(d: int, s: float):
    """uint64 thresholds T[r] = floor(2^64 * P(rank <= r)) for ranks 0..d-1,
    P(rank = r) proportional to (r+1)^-s.  The last threshold is 2^64-1."""
    w = np.arange(1, d + 1, dtype=np.float64) ** (-float(s))
    c = np.cumsum(w)
    c /= c[-1]
    t = np.floor(c * 18446744073709551616.0)
    t = np.minimum(t, 18446744073709549568.0)  # largest double below 2^64
    out = t.astype(np.uint64)
    out[-1] = np.uint64(0xFFFFFFFFFFFFFFFF)
    return out


def zipf_ranks(seed: int, n: int, d: int, s: float, start: int = 0, table=None):
    """n ranks in [0, d) with P(r) proportional to (r+1)^-s (s=0 is uniform)."""
    if s == 0:
        return uniform_ranks(seed, n, d, start)
    if table is None:
        table = zipf_cdf_table(d, s)
    u = stream(seed, start, n)
    r = np.searchsorted(table, u, side="left").astype(np.uint64)
    return np.minimum(r, np.uint64(d - 1))


def uniform_i64(seed: int, n: int, lo: int = -1_000_000, hi: int = 1_000_000, start: int = 0):
    """n int64 values uniform over [lo, hi]."""
    span = hi - lo + 1
    return mulhi64(stream(seed, start, n), span).astype(np.int64) + np.int64(lo)


def normal_f64(seed: int, n: int):
    """n standard-normal float64 values (numpy PCG64 seeded with ``seed``)."""
    return np.random.Generator(np.random.PCG64(seed)).standard_normal(n)


def plain_input(seed: int, n: int, d: int, s: float = 0.0, with_f64: bool = False,
                table=None):
    """A group-by input: uint64 keys over a d-value domain (uniform or Zipf s),
    int64 values uniform in [-1e6, 1e6], optionally float64 N(0,1) values.
    Three independent sub-streams of the master seed."""
    ranks = zipf_ranks(substream_seed(seed, 1), n, d, s, table=table)
    keys = key_of_rank(ranks)
    v = uniform_i64(substream_seed(seed, 2), n)
    f = normal_f64(substream_seed(seed, 3) & 0xFFFFFFFF, n) if with_f64 else None
    return keys, v, f


def segmented_input(seed: int, n: int, n_a: int = 1000, b_per_a: int = 100_000):
    """Composite-key input sorted on A only: A takes n_a distinct random int32
    values (ascending, rows assigned uniformly at random, then sorted), B is
    drawn per row uniformly from a per-A domain of b_per_a random int32 values
    (both signs), unsorted within a segment; v is int64 uniform in [-1e6,1e6]."""
    cand = (stream(substream_seed(seed, 10), 0, 4 * n_a) >> np.uint64(32)).astype(np.uint32).view(np.int32)
    _, first = np.unique(cand, return_index=True)
    a_vals = np.sort(cand[np.sort(first)[:n_a]])
    n_a = a_vals.shape[0]
    seg = np.sort(mulhi64(stream(substream_seed(seed, 11), 0, n), n_a).astype(np.int64))
    a = a_vals[seg]
    # B: per-A domain value j of segment g is the top 32 bits of mix(g*b_per_a + j)
    j = mulhi64(stream(substream_seed(seed, 12), 0, n), b_per_a).astype(np.uint64)
    code = seg.astype(np.uint64) * np.uint64(b_per_a) + j
    b = (mix64(code ^ np.uint64(substream_seed(seed, 13))) >> np.uint64(32)).astype(np.uint32).view(np.int32)
    v = uniform_i64(substream_seed(seed, 14), n)
    return a, b, v

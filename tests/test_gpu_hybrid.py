"""GPU parity of hybrid run generation (Section 5, hybrid algorithms): a
resident index keeps the key values below a cut in memory for good, the other
key values go to runs by read-sort-write cycles, and both indexes join the
final wide merge.  The grouped output equals the oracle's (integers bit-exact,
the fp64 sum within 1e-12 * sum |x|), and the run count and spilled rows equal
the batch-granular hybrid simulator's for the capacities the call reports."""
import numpy as np
import pytest

import datagen
from oracle import spillsim
import paper_2010_00152_amd as isa
from tests.gpu_util import compare, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = isa.Context(0)
    c.set_run_generation(isa.ISA_RUNGEN_HYBRID)
    yield c
    c.close()


def _sim(k, st):
    return spillsim.simulate_hybrid(k, st["batch_rows"], st["resident_capacity"], st["run_capacity"])


@pytest.mark.parametrize("s,seed,budget_mib,share", [(0.0, 5, 16, 800), (0.8, 6, 16, 800), (1.2, 7, 16, 800),
                                                     (0.8, 6, 20, 500), (0.0, 8, 24, 650)])
def test_hybrid_matches_oracle_and_simulator(ctx, s, seed, budget_mib, share):
    say("case hybrid s=%s budget=%dMiB share=%d" % (s, budget_mib, share))
    ctx.set_resident_share(share)
    n = 1_500_000
    k, v, f = datagen.plain_input(seed, n, 400_000, s, with_f64=True)
    got, st, status, g = run_gpu(ctx, k, v, f, budget=budget_mib << 20)
    compare(got, k, v, f, isa.ISA_ALL, "hybrid")
    assert st["resident_capacity"] > 0 and st["run_capacity"] >= st["batch_rows"]
    sim = _sim(k, st)
    assert st["runs"] == sim["runs"] and st["spilled_rows"] == sim["spilled_rows"], (st, sim)
    assert st["spilled_rows"] <= n and st["peak_ws_bytes"] <= budget_mib << 20
    if s < 1.2:
        assert "demotion" in sim["run_kinds"] and st["windows"] >= 1


def test_hybrid_without_resident_share_is_read_sort_write(ctx):
    # a share of 0: every key goes to runs; the spill statistics are those of
    # read-sort-write cycles with the run-generation index's capacity
    say("case hybrid share 0")
    ctx.set_resident_share(0)
    k, v, _ = datagen.plain_input(9, 1_200_000, 300_000, 0.3)
    got, st, status, g = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=24 << 20)
    compare(got, k, v, None, isa.ISA_INT_AGGS, "hybrid share 0")
    assert st["resident_capacity"] == 0
    sim = spillsim.simulate(k, st["batch_rows"], st["run_capacity"])
    assert st["runs"] == sim["runs"] > 0 and st["spilled_rows"] == sim["spilled_rows"]
    ctx.set_resident_share(800)


def test_hybrid_same_output_as_read_sort_write_and_resident_absorbs(ctx):
    # the policy changes spilling, never the integer output; with a skewed
    # input the resident index keeps the smallest keys in memory for good
    say("case hybrid vs read-sort-write")
    ctx.set_resident_share(800)
    k, v, _ = datagen.plain_input(44, 1_200_000, 600_000, 0.6)
    got_h, st_h, _, g_h = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20)
    ctx.set_run_generation(isa.ISA_RUNGEN_READ_SORT_WRITE)
    try:
        got_w, st_w, _, g_w = run_gpu(ctx, k, v, None, aggs=isa.ISA_INT_AGGS, budget=16 << 20)
    finally:
        ctx.set_run_generation(isa.ISA_RUNGEN_HYBRID)
    assert g_h == g_w
    for c in got_w:
        assert np.array_equal(got_h[c], got_w[c]), c
    sim = _sim(k, st_h)
    assert st_h["runs"] == sim["runs"] and st_h["spilled_rows"] == sim["spilled_rows"]
    assert sim["resident_rows"] > 0 and sim["cut"] < 1 << 64
    with pytest.raises(isa.InsortError):
        ctx.set_resident_share(1001)

"""The entry point for callers that cannot allocate (isa_group_by_noalloc),
called through the C ABI: its output equals isa_group_by's on the same input
(integer columns bit-exact, the fp64 sum within 1e-12 * sum |x| per group; the
same kernels run, so in practice identical), on two calls in a row whose
second input is smaller, so that what the first call left in the shared
scratch must not leak into the second."""
import ctypes

import numpy as np
import pytest

import datagen
import paper_2010_00152_amd as isa
from tests.gpu_util import FP64_REL, compare, say, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = isa.Context(0)
    yield c
    c.close()


def _call(ctx, fn, kd, vd, fd, aggs, cap):
    import torch
    n = kd.numel()
    o = isa._alloc_outputs(torch, cap, aggs, "cuda")
    out = isa._output_struct(o, cap)
    inp = isa.isa_input(isa._ptr(kd), isa._ptr(vd), isa._ptr(fd), n)
    sp = isa._stream_ptr()
    L = isa.lib()
    if fn == "noalloc":
        st = L.isa_group_by_noalloc(ctx.handle, ctypes.byref(inp), aggs, ctypes.byref(out), sp)
    else:
        ws = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        st = L.isa_group_by(ctx.handle, ctypes.byref(inp), aggs, isa.isa_workspace(isa._ptr(ws), ws.numel()),
                            isa.isa_spill(None, 0), ctypes.byref(out), None, sp)
    torch.cuda.synchronize()
    g = out.n_groups
    res = {}
    for c, t in o.items():
        dt = {"keys": np.uint64, "count": np.uint64, "sum_f64": np.float64}.get(c, np.int64)
        res[c] = to_np(t[:g], dt)
    return st, g, res


@pytest.mark.parametrize("aggs", [isa.ISA_ALL, isa.ISA_INT_AGGS])
def test_noalloc_equals_group_by_on_two_calls(ctx, aggs):
    L = isa.lib()
    nmax = L.isa_noalloc_max_rows(aggs)
    assert nmax > 1_000_000
    # first a large input near the limit (all of it), then a smaller one with
    # fewer groups and a ragged size
    for seed, n, d, s in [(71, nmax, 400_000, 0.6), (72, 123_457, 5_000, 0.0)]:
        say("case noalloc aggs=%d n=%d d=%d" % (aggs, n, d))
        k, v, f = datagen.plain_input(seed, n, d, s, with_f64=True)
        kd, vd, fd = to_dev(k), to_dev(v), to_dev(f)
        if not aggs & isa.ISA_SUM_F64:
            fd = f = None
        st_a, g_a, got = _call(ctx, "noalloc", kd, vd, fd, aggs, min(n, d))
        st_b, g_b, ref = _call(ctx, "group_by", kd, vd, fd, aggs, min(n, d))
        assert st_a == isa.ISA_OK and st_b == isa.ISA_OK, (st_a, st_b, ctx.last_error())
        assert g_a == g_b
        for c in ref:
            if c == "sum_f64":
                absum = isa_abs_sum(k, f)
                assert (np.abs(got[c] - ref[c]) <= FP64_REL * absum).all()
            else:
                assert np.array_equal(got[c], ref[c]), c
        compare(got, k, v, f, aggs, "noalloc n=%d" % n)


def isa_abs_sum(k, f):
    import oracle
    return oracle.group_by(k, None, np.abs(f))["sum_f64"]


def test_noalloc_rejects_beyond_its_scratch(ctx):
    import torch
    L = isa.lib()
    n = L.isa_noalloc_max_rows(isa.ISA_INT_AGGS) + 1
    k = torch.zeros(n, dtype=torch.int64, device="cuda")
    o = isa._alloc_outputs(torch, 16, isa.ISA_INT_AGGS, "cuda")
    out = isa._output_struct(o, 16)
    inp = isa.isa_input(isa._ptr(k), isa._ptr(k), None, n)
    st = L.isa_group_by_noalloc(ctx.handle, ctypes.byref(inp), isa.ISA_INT_AGGS, ctypes.byref(out),
                                isa._stream_ptr())
    assert st == isa.ISA_EBUDGET and out.n_groups == 0
    # empty input: nothing to do
    inp0 = isa.isa_input(isa._ptr(k), isa._ptr(k), None, 0)
    assert L.isa_group_by_noalloc(ctx.handle, ctypes.byref(inp0), isa.ISA_INT_AGGS, ctypes.byref(out),
                                  isa._stream_ptr()) == isa.ISA_OK
    # a missing column for a requested aggregate
    inp1 = isa.isa_input(isa._ptr(k), None, None, 10)
    assert L.isa_group_by_noalloc(ctx.handle, ctypes.byref(inp1), isa.ISA_INT_AGGS, ctypes.byref(out),
                                  isa._stream_ptr()) == isa.ISA_EINVAL

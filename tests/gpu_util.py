"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and compare with the CPU oracle on the same seeded inputs."""
import math
import sys

import numpy as np

import oracle
import paper_2010_00152_amd as isa

# fp64 sum tolerance per group: |gpu - exact| <= FP64_REL * sum(|x|) over the group
FP64_REL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    if a is None:
        return None
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def to_np(t, dtype):
    a = t.cpu().numpy()
    return a.view(dtype) if a.dtype != dtype else a


def run_gpu(ctx, keys, v=None, f=None, aggs=isa.ISA_ALL, budget=256 << 20, capacity=None,
            spill_bytes=None, check=True):
    import torch
    kd, vd, fd = to_dev(keys), to_dev(v), to_dev(f)
    res, stats, status, g = isa.group_by(ctx, kd, vd, fd, aggs=aggs, mem_budget=budget,
                                         capacity=capacity, spill_bytes=spill_bytes, check=check)
    torch.cuda.synchronize()
    out = {}
    for k, t in res.items():
        dt = {"keys": np.uint64, "count": np.uint64, "sum_f64": np.float64}.get(k, np.int64)
        out[k] = to_np(t, dt)
    return out, stats, status, g


def compare(got, keys, v, f, aggs, label=""):
    """Element-by-element comparison with the oracle: integer columns bit-exact,
    the fp64 sum within FP64_REL * sum(|x|) per group."""
    ref = oracle.group_by(keys, v, f)
    assert got["keys"].shape == ref["keys"].shape, (label, got["keys"].shape, ref["keys"].shape)
    assert np.array_equal(got["keys"], ref["keys"]), label
    if aggs & isa.ISA_COUNT:
        assert np.array_equal(got["count"], ref["count"]), label
    if aggs & isa.ISA_SUM_I64:
        assert np.array_equal(got["sum_i64"], ref["sum_i64"]), label
    if aggs & isa.ISA_MIN_I64:
        assert np.array_equal(got["min_i64"], ref["min_i64"]), label
    if aggs & isa.ISA_MAX_I64:
        assert np.array_equal(got["max_i64"], ref["max_i64"]), label
    if aggs & isa.ISA_SUM_F64:
        absum = oracle.group_by(keys, None, np.abs(f))["sum_f64"]
        err = np.abs(got["sum_f64"] - ref["sum_f64"])
        bad = err > FP64_REL * absum
        assert not bad.any(), (label, int(bad.sum()), float((err / np.maximum(absum, 1e-300)).max()))
    return ref

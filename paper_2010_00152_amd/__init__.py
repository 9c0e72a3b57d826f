"""Python binding of libinsort.so: sort-based duplicate removal, grouping and
aggregation on AMD MI355X (gfx950).

The C ABI (include/insort.h) is exposed under the same names (``isa_*``);
this module only marshals arguments.  Every step of the grouping runs in the
library's HIP kernels; PyTorch is used to allocate device and pinned memory
and to name streams.  There is no fallback: if the library is missing or the
device is not a gfx950 GPU, calls raise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libinsort.so")

ISA_OK = 0
ISA_EINVAL = -1
ISA_EBUDGET = -2
ISA_ESPILL = -3
ISA_ETRUNC = -4
ISA_EDEVICE = -5
ISA_ENOMEM = -6
ISA_EUNIMPL = -7
ISA_EBUSY = -8

ISA_COUNT = 1
ISA_SUM_I64 = 2
ISA_SUM_F64 = 4
ISA_MIN_I64 = 8
ISA_MAX_I64 = 16
ISA_ALL = ISA_COUNT | ISA_SUM_I64 | ISA_SUM_F64 | ISA_MIN_I64 | ISA_MAX_I64
ISA_INT_AGGS = ISA_COUNT | ISA_SUM_I64 | ISA_MIN_I64 | ISA_MAX_I64
ISA_RUNGEN_READ_SORT_WRITE = 0
ISA_RUNGEN_REPLACEMENT = 1
ISA_RUNGEN_HYBRID = 2

P = ctypes.c_void_p
U64 = ctypes.c_uint64
U32 = ctypes.c_uint32


class isa_input(ctypes.Structure):
    _fields_ = [("keys", P), ("v_i64", P), ("v_f64", P), ("n_rows", U64)]


class isa_output(ctypes.Structure):
    _fields_ = [("keys", P), ("count", P), ("sum_i64", P), ("sum_f64", P),
                ("min_i64", P), ("max_i64", P), ("capacity", U64), ("n_groups", U64)]


class isa_workspace(ctypes.Structure):
    _fields_ = [("dev", P), ("bytes", U64)]


class isa_spill(ctypes.Structure):
    _fields_ = [("host_pinned", P), ("bytes", U64)]


class isa_stats(ctypes.Structure):
    _fields_ = [("runs", U64), ("spilled_rows", U64), ("spilled_bytes", U64), ("windows", U64),
                ("batches", U64), ("index_capacity", U64), ("batch_rows", U64),
                ("peak_ws_bytes", U64), ("t_rungen_ms", ctypes.c_double),
                ("t_merge_ms", ctypes.c_double), ("t_plan_ms", ctypes.c_double),
                ("merge_steps", U64), ("merge_rows", U64), ("resident_capacity", U64),
                ("run_capacity", U64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class isa_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", U64), ("rows", U64), ("bytes", U64),
                ("total_ms", ctypes.c_double)]


class isa_tuning(ctypes.Structure):
    _fields_ = [("leaf_rows", U32), ("chunk_split", U32), ("graph", U32), ("merge_fanin", U32)]

    def as_dict(self):
        return {"leaf_rows": self.leaf_rows, "chunk_split": self.chunk_split, "graph": self.graph,
                "merge_fanin": self.merge_fanin}


# Every function the header declares: name -> (restype, argtypes)
SIGNATURES = {
    "isa_ctx_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(P)]),
    "isa_ctx_destroy": (None, [P]),
    "isa_state_row_bytes": (U64, [U32]),
    "isa_min_workspace_bytes": (U64, [U32]),
    "isa_group_by": (ctypes.c_int, [P, ctypes.POINTER(isa_input), U32, isa_workspace, isa_spill,
                                    ctypes.POINTER(isa_output), ctypes.POINTER(isa_stats), P]),
    "isa_group_by_noalloc": (ctypes.c_int, [P, ctypes.POINTER(isa_input), U32, ctypes.POINTER(isa_output), P]),
    "isa_noalloc_max_rows": (U64, [U32]),
    "isa_group_by_columns": (ctypes.c_int, [P, ctypes.POINTER(P), U32, P, U64, U32, isa_workspace,
                                            ctypes.POINTER(P), ctypes.POINTER(isa_output), P, P,
                                            ctypes.POINTER(U64), P]),
    "isa_columns_workspace_bytes": (U64, [U64, U32]),
    "isa_group_by_segmented": (ctypes.c_int, [P, P, P, P, U64, U32, isa_workspace, P, P,
                                              ctypes.POINTER(isa_output), P]),
    "isa_group_by_sorted": (ctypes.c_int, [P, ctypes.POINTER(isa_input), U32, isa_workspace,
                                           ctypes.POINTER(isa_output), P]),
    "isa_count_distinct": (ctypes.c_int, [P, P, P, U64, isa_workspace, isa_spill, P, U64, P, P, P, U64,
                                          ctypes.POINTER(U64), P]),
    "isa_batch_run": (ctypes.c_int, [P, U32, ctypes.POINTER(isa_input), U32, isa_workspace,
                                     ctypes.POINTER(isa_output), P]),
    "isa_batch_workspace_bytes": (U64, [U32, ctypes.POINTER(isa_input), U32]),
    "isa_server_create": (ctypes.c_int, [P, P, U64, U32, ctypes.POINTER(P)]),
    "isa_server_submit": (ctypes.c_int, [P, ctypes.POINTER(isa_input), U32,
                                         ctypes.POINTER(isa_output), ctypes.POINTER(U64)]),
    "isa_server_poll": (ctypes.c_int, [P, U64, ctypes.POINTER(ctypes.c_int),
                                       ctypes.POINTER(ctypes.c_double)]),
    "isa_server_drain": (ctypes.c_int, [P]),
    "isa_server_release": (ctypes.c_int, [P, U64]),
    "isa_server_destroy": (None, [P]),
    "isa_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "isa_last_error": (ctypes.c_char_p, [P]),
    "isa_profile_enable": (ctypes.c_int, [P, ctypes.c_int]),
    "isa_profile_read": (ctypes.c_int, [P, ctypes.POINTER(isa_kernel_time), ctypes.c_int]),
    "isa_set_run_generation": (ctypes.c_int, [P, ctypes.c_int]),
    "isa_get_run_generation": (ctypes.c_int, [P]),
    "isa_set_resident_share": (ctypes.c_int, [P, U32]),
    "isa_get_tuning": (ctypes.c_int, [P, ctypes.POINTER(isa_tuning)]),
    "isa_set_tuning": (ctypes.c_int, [P, ctypes.POINTER(isa_tuning)]),
    "isa_tune_candidates": (U32, [ctypes.POINTER(isa_tuning), U32]),
    "isa_tune_batch": (ctypes.c_int, [P, U32, ctypes.POINTER(isa_input), U32, isa_workspace,
                                      ctypes.POINTER(isa_output), P, ctypes.POINTER(isa_tuning),
                                      ctypes.POINTER(ctypes.c_double), U32]),
}

_lib = None


def lib():
    """Load libinsort.so (raises if it was not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libinsort.so is not built; run paper_2010_00152_amd/build.py")
        # torch's HIP runtime must be the one the library binds to: loaded
        # first, it satisfies the library's libamdhip64 dependency; loaded
        # after, a second runtime would come up without the GPU
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class InsortError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s (%d)%s" % (lib().isa_status_str(status).decode(), status,
                                        (": " + msg) if msg else ""))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Context:
    """A library context bound to one GPU."""

    def __init__(self, device: int = 0):
        h = P()
        st = lib().isa_ctx_create(device, ctypes.byref(h))
        if st != ISA_OK:
            raise InsortError(st, "isa_ctx_create(%d)" % device)
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            lib().isa_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def last_error(self) -> str:
        return lib().isa_last_error(self.handle).decode()

    def profile(self, on: bool = True):
        st = lib().isa_profile_enable(self.handle, 1 if on else 0)
        if st != ISA_OK:
            raise InsortError(st)

    def set_run_generation(self, policy: int):
        """ISA_RUNGEN_READ_SORT_WRITE or ISA_RUNGEN_REPLACEMENT (isa_set_run_generation)."""
        st = lib().isa_set_run_generation(self.handle, policy)
        if st != ISA_OK:
            raise InsortError(st, self.last_error())

    def set_resident_share(self, permille: int):
        st = lib().isa_set_resident_share(self.handle, permille)
        if st != ISA_OK:
            raise InsortError(st, self.last_error())

    def get_run_generation(self) -> int:
        return lib().isa_get_run_generation(self.handle)

    def get_tuning(self) -> dict:
        t = isa_tuning()
        st = lib().isa_get_tuning(self.handle, ctypes.byref(t))
        if st != ISA_OK:
            raise InsortError(st)
        return t.as_dict()

    @staticmethod
    def default_tuning() -> dict:
        """The launch configuration a new context starts with."""
        return {"leaf_rows": 2048, "chunk_split": 512, "graph": 1, "merge_fanin": 0}

    def set_tuning(self, leaf_rows: int = 2048, chunk_split: int = 512, graph: int = 1, merge_fanin: int = 0):
        t = isa_tuning(leaf_rows, chunk_split, graph, merge_fanin)
        st = lib().isa_set_tuning(self.handle, ctypes.byref(t))
        if st != ISA_OK:
            raise InsortError(st, "tuning %r" % (t.as_dict(),))

    def profile_read(self):
        """{name: {launches, rows, bytes, total_ms}} of launches since profile(True)."""
        buf = (isa_kernel_time * 64)()
        n = lib().isa_profile_read(self.handle, buf, 64)
        if n < 0:
            raise InsortError(n)
        return {buf[i].name.decode(): {"launches": buf[i].launches, "rows": buf[i].rows,
                                       "bytes": buf[i].bytes, "total_ms": buf[i].total_ms}
                for i in range(min(n, 64))}


def _alloc_outputs(torch, cap, aggs, dev, with_keys=True):
    o = {}
    if with_keys:
        o["keys"] = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)  # uint64 bits
    if aggs & ISA_COUNT:
        o["count"] = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)  # uint64 bits
    if aggs & ISA_SUM_I64:
        o["sum_i64"] = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    if aggs & ISA_SUM_F64:
        o["sum_f64"] = torch.empty(max(cap, 1), dtype=torch.float64, device=dev)
    if aggs & ISA_MIN_I64:
        o["min_i64"] = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    if aggs & ISA_MAX_I64:
        o["max_i64"] = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    return o


def _output_struct(o, cap):
    return isa_output(_ptr(o.get("keys")), _ptr(o.get("count")), _ptr(o.get("sum_i64")),
                      _ptr(o.get("sum_f64")), _ptr(o.get("min_i64")), _ptr(o.get("max_i64")),
                      cap, 0)


def group_by(ctx: Context, keys, v_i64=None, v_f64=None, aggs: int = ISA_ALL,
             mem_budget: int = 256 << 20, capacity: int | None = None, spill_bytes: int | None = None,
             workspace=None, spill=None, stream=None, check: bool = True):
    """group_by(keys, values, aggs, mem_budget) -> sorted (key, count, sum, min, max).

    keys: CUDA tensor of uint64 key bits (int64 or uint64 dtype); v_i64: int64;
    v_f64: float64 (same length).  Output keys and counts are int64 tensors
    holding uint64 bits.
    Returns (dict of output tensors trimmed to n_groups, stats dict, status)."""
    import torch
    dev = keys.device
    n = keys.numel()
    cap = n if capacity is None else capacity
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device=dev)
    if spill is None:
        sb = spill_bytes if spill_bytes is not None else n * lib().isa_state_row_bytes(aggs)
        spill = torch.empty(max(sb, 1), dtype=torch.uint8, pin_memory=True) if sb else None
    o = _alloc_outputs(torch, cap, aggs, dev)
    out = _output_struct(o, cap)
    inp = isa_input(_ptr(keys), _ptr(v_i64), _ptr(v_f64), n)
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    sp = isa_spill(_ptr(spill), spill.numel() if spill is not None else 0)
    st = isa_stats()
    status = lib().isa_group_by(ctx.handle, ctypes.byref(inp), aggs, ws, sp, ctypes.byref(out),
                                ctypes.byref(st), _stream_ptr(stream))
    if check and status not in (ISA_OK,):
        raise InsortError(status, ctx.last_error())
    g = out.n_groups
    res = {k: v[:min(g, cap)] for k, v in o.items()}
    return res, st.as_dict(), status, g


def group_by_sorted(ctx: Context, keys, v_i64=None, v_f64=None, aggs: int = ISA_ALL, mem_budget: int = 16 << 20,
                    capacity: int | None = None, workspace=None, stream=None, check: bool = True):
    """Group input already sorted on its key (isa_group_by_sorted).
    Returns (dict of output tensors trimmed to n_groups, status, n_groups)."""
    import torch
    dev = keys.device
    n = keys.numel()
    cap = n if capacity is None else capacity
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device=dev)
    o = _alloc_outputs(torch, cap, aggs, dev)
    out = _output_struct(o, cap)
    inp = isa_input(_ptr(keys), _ptr(v_i64), _ptr(v_f64), n)
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    status = lib().isa_group_by_sorted(ctx.handle, ctypes.byref(inp), aggs, ws, ctypes.byref(out),
                                       _stream_ptr(stream))
    if check and status != ISA_OK:
        raise InsortError(status, ctx.last_error())
    g = out.n_groups
    return {k: v[:min(g, cap)] for k, v in o.items()}, status, g


def count_distinct(ctx: Context, g, x, mem_budget: int = 256 << 20, capacity: int | None = None,
                   spill_bytes: int | None = None, workspace=None, scratch=None, stream=None, check: bool = True):
    """count(*) and count(distinct x) per g for int32 CUDA tensors g, x
    (isa_count_distinct).  Returns (dict g/count/distinct trimmed to
    n_groups, status, n_groups)."""
    import torch
    dev = g.device
    n = g.numel()
    cap = n if capacity is None else capacity
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device=dev)
    if scratch is None:
        scratch = torch.empty(max(24 * n, 8), dtype=torch.uint8, device=dev)
    sb = spill_bytes if spill_bytes is not None else n * lib().isa_state_row_bytes(ISA_COUNT)
    spill = torch.empty(max(sb, 1), dtype=torch.uint8, pin_memory=True) if sb else None
    og = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    oc = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    od = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
    ng = U64()
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    sp = isa_spill(_ptr(spill), spill.numel() if spill is not None else 0)
    status = lib().isa_count_distinct(ctx.handle, _ptr(g), _ptr(x), n, ws, sp, _ptr(scratch), scratch.numel(),
                                      _ptr(og), _ptr(oc), _ptr(od), cap, ctypes.byref(ng), _stream_ptr(stream))
    if check and status != ISA_OK:
        raise InsortError(status, ctx.last_error())
    k = min(ng.value, cap)
    return {"g": og[:k], "count": oc[:k], "distinct": od[:k]}, status, ng.value


def group_by_columns(ctx: Context, cols, v=None, aggs: int = ISA_COUNT | ISA_SUM_I64, mem_budget: int | None = None,
                     capacity: int | None = None, codes: bool = False, check: bool = True, workspace=None):
    """isa_group_by_columns: group on the int64 columns `cols` (device tensors
    of equal length).  Returns (result dict with "cols" (list of key columns)
    and the aggregate columns, codes dict or None, column compares, status,
    n_groups)."""
    import torch
    K = len(cols)
    n = cols[0].numel()
    dev = cols[0].device
    cap = n if capacity is None else capacity
    need = lib().isa_columns_workspace_bytes(n, K)
    budget = need if mem_budget is None else mem_budget
    ws = workspace if workspace is not None else torch.empty(max(budget, 256), dtype=torch.uint8, device=dev)
    o = _alloc_outputs(torch, cap, aggs, dev, with_keys=False)
    outc = [torch.empty(max(cap, 1), dtype=torch.int64, device=dev) for _ in range(K)]
    out = _output_struct(o, cap)
    kin = (P * K)(*[_ptr(c) for c in cols])
    kout = (P * K)(*[_ptr(c) for c in outc])
    co = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if codes else None
    cv = torch.empty(max(n, 1), dtype=torch.int64, device=dev) if codes else None
    cmp = U64()
    st = lib().isa_group_by_columns(ctx.handle, kin, K, _ptr(v), n, aggs, isa_workspace(_ptr(ws), budget), kout,
                                    ctypes.byref(out), _ptr(co), _ptr(cv), ctypes.byref(cmp), _stream_ptr())
    if check and st not in (ISA_OK, ISA_ETRUNC):
        raise InsortError(st, ctx.last_error())
    g = out.n_groups
    k = min(g, cap)
    res = {c: t[:k] for c, t in o.items()}
    res["cols"] = [c[:k] for c in outc]
    cd = {"offset": co[:n], "value": cv[:n]} if codes else None
    return res, cd, cmp.value, st, g


def group_by_segmented(ctx: Context, a, b, v=None, aggs: int = ISA_INT_AGGS, mem_budget: int = 256 << 20,
                       capacity: int | None = None, workspace=None, stream=None, check: bool = True):
    """Group on (a, b) for input sorted on a (int32 CUDA tensors; v int64).
    Returns (dict with a, b and the aggregate columns, status, n_groups)."""
    import torch
    dev = a.device
    n = a.numel()
    cap = n if capacity is None else capacity
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device=dev)
    o = _alloc_outputs(torch, cap, aggs, dev, with_keys=False)
    oa = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    ob = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    out = _output_struct(o, cap)
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    status = lib().isa_group_by_segmented(ctx.handle, _ptr(a), _ptr(b), _ptr(v), n, aggs, ws, _ptr(oa),
                                          _ptr(ob), ctypes.byref(out), _stream_ptr(stream))
    if check and status != ISA_OK:
        raise InsortError(status, ctx.last_error())
    g = out.n_groups
    m = min(g, cap)
    res = {k: t[:m] for k, t in o.items()}
    res["a"] = oa[:m]
    res["b"] = ob[:m]
    return res, status, g


def batch_run(ctx: Context, inputs, aggs: int = ISA_INT_AGGS, mem_budget: int = 1 << 30, workspace=None,
              stream=None, check: bool = True):
    """Run many independent group-bys together.  inputs: list of (keys, v_i64, v_f64)
    CUDA tensors (v_* may be None).  Returns (list of output dicts, status)."""
    import torch
    k = len(inputs)
    ins = (isa_input * max(k, 1))()
    outs = (isa_output * max(k, 1))()
    keep = []
    for i, (kk, vv, ff) in enumerate(inputs):
        n = kk.numel()
        o = _alloc_outputs(torch, n, aggs, kk.device)
        keep.append(o)
        ins[i] = isa_input(_ptr(kk), _ptr(vv), _ptr(ff), n)
        outs[i] = _output_struct(o, n)
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device="cuda")
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    status = lib().isa_batch_run(ctx.handle, k, ins, aggs, ws, outs, _stream_ptr(stream))
    if check and status != ISA_OK:
        raise InsortError(status, ctx.last_error())
    res = []
    for i in range(k):
        g = outs[i].n_groups
        res.append({c: t[:g] for c, t in keep[i].items()})
    return res, status


def tune_candidates():
    n = lib().isa_tune_candidates(None, 0)
    buf = (isa_tuning * n)()
    lib().isa_tune_candidates(buf, n)
    return [buf[i].as_dict() for i in range(n)]


def tune_batch(ctx: Context, inputs, aggs: int = ISA_INT_AGGS, mem_budget: int = 1 << 30, workspace=None,
               stream=None):
    """Autotune the launch configuration on a batch of instances (list of
    (keys, v_i64, v_f64) CUDA tensors); the fastest configuration stays set on
    the context.  Returns (best config dict, {candidate index: ms})."""
    import torch
    k = len(inputs)
    ins = (isa_input * max(k, 1))()
    outs = (isa_output * max(k, 1))()
    keep = []
    for i, (kk, vv, ff) in enumerate(inputs):
        n = kk.numel()
        o = _alloc_outputs(torch, n, aggs, kk.device)
        keep.append(o)
        ins[i] = isa_input(_ptr(kk), _ptr(vv), _ptr(ff), n)
        outs[i] = _output_struct(o, n)
    if workspace is None:
        workspace = torch.empty(mem_budget, dtype=torch.uint8, device="cuda")
    ws = isa_workspace(_ptr(workspace), workspace.numel())
    nc = lib().isa_tune_candidates(None, 0)
    times = (ctypes.c_double * nc)()
    best = isa_tuning()
    st = lib().isa_tune_batch(ctx.handle, k, ins, aggs, ws, outs, _stream_ptr(stream), ctypes.byref(best), times, nc)
    if st != ISA_OK:
        raise InsortError(st, ctx.last_error())
    return best.as_dict(), {i: times[i] for i in range(nc)}


class Server:
    """Continuous-batching request loop of the library (isa_server_*).  Inputs
    must be ready on the device when submitted; keep them alive until done."""

    def __init__(self, ctx: Context, cap_bytes: int, slots: int = 2, workspace=None):
        import torch
        self.ctx = ctx
        self.workspace = workspace if workspace is not None else torch.empty(
            cap_bytes, dtype=torch.uint8, device="cuda")
        h = P()
        st = lib().isa_server_create(ctx.handle, _ptr(self.workspace), cap_bytes, slots, ctypes.byref(h))
        if st != ISA_OK:
            raise InsortError(st)
        self.handle = h
        self.live = {}

    def submit(self, keys, v_i64=None, v_f64=None, aggs: int = ISA_INT_AGGS, capacity: int | None = None):
        import torch
        n = keys.numel()
        cap = n if capacity is None else capacity
        o = _alloc_outputs(torch, cap, aggs, keys.device)
        out = _output_struct(o, cap)
        inp = isa_input(_ptr(keys), _ptr(v_i64), _ptr(v_f64), n)
        t = U64()
        st = lib().isa_server_submit(self.handle, ctypes.byref(inp), aggs, ctypes.byref(out), ctypes.byref(t))
        if st != ISA_OK:
            raise InsortError(st)
        self.live[t.value] = (keys, v_i64, v_f64, o, out, inp)
        return t.value

    def poll(self, ticket):
        done = ctypes.c_int()
        lat = ctypes.c_double()
        st = lib().isa_server_poll(self.handle, ticket, ctypes.byref(done), ctypes.byref(lat))
        return bool(done.value), lat.value, st

    def result(self, ticket):
        _, _, _, o, out, _ = self.live[ticket]
        g = out.n_groups
        return {c: t[:g] for c, t in o.items()}

    def release(self, ticket):
        """Forget a finished request (isa_server_release) and return its result
        columns; the binding drops its references to the request's buffers."""
        st = lib().isa_server_release(self.handle, ticket)
        if st != ISA_OK:
            raise InsortError(st)
        res = self.result(ticket)
        del self.live[ticket]
        return res

    def drain(self):
        st = lib().isa_server_drain(self.handle)
        if st != ISA_OK:
            raise InsortError(st)

    def close(self):
        if self.handle:
            lib().isa_server_destroy(self.handle)
            self.handle = None

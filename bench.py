"""Benchmark: sort-based grouping with early aggregation and wide merging on one
MI355X.

A step is one full group-by over one synthetic input resident in HBM: run
generation (batch sort, absorb into the index, spill runs to pinned host
memory) and the wide merge into sorted output.  Default workload: 100M rows,
uint64 keys over 1e7 values with Zipf skew 0.8, int64 value and float64 value,
count/sum(int64)/sum(fp64)/min/max, workspace budget 256 MiB.

Prints one JSON line (see the keys below).  --gpus N with N > 1 exits: this
build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth

WORKLOADS = {
    # name: (rows, distinct domain, zipf s, seed, budget MiB, with f64, aggs name)
    "spill_100M_zipf0.8": (100_000_000, 10_000_000, 0.8, 3, 256, True, "all"),
    "spill_100M_zipf0": (100_000_000, 10_000_000, 0.0, 2, 256, True, "all"),
    "spill_100M_zipf1.2": (100_000_000, 10_000_000, 1.2, 4, 256, True, "all"),
    "nospill_100M_zipf0.8": (100_000_000, 10_000_000, 0.8, 3, 12 * 1024, True, "all"),
    "nospill_100M_zipf0": (100_000_000, 10_000_000, 0.0, 2, 12 * 1024, True, "all"),
    "nospill_100M_zipf1.2": (100_000_000, 10_000_000, 1.2, 4, 12 * 1024, True, "all"),
    "plain_1M_10k": (1_000_000, 10_000, 0.0, 1, 64, False, "int"),
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spill_100M_zipf0.8", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="rows of the input the CPU oracle is timed on (0 = skip)")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (--gpus %d requested); "
              "multi-GPU sharding is a design note, not built" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": nbytes, "calibrate_copy_bytes_written": nbytes,
                          "launches": 3}))
        return

    import datagen
    import datagen.device as dgd
    import paper_2010_00152_amd as isa

    n, d, s, seed, budget_mib, with_f, aggs_name = WORKLOADS[args.workload]
    aggs = isa.ISA_ALL if aggs_name == "all" else isa.ISA_INT_AGGS
    print("bench: workload %s, generating %d rows on the device" % (args.workload, n), file=sys.stderr,
          flush=True)
    kd, vd, fd = dgd.plain_input(seed, n, d, s, with_f64=with_f)
    torch.cuda.synchronize()
    ctx = isa.Context(0)
    L = isa.lib()
    budget = budget_mib << 20
    ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
    row_b = L.isa_state_row_bytes(aggs)
    spill = torch.empty(n * row_b, dtype=torch.uint8, pin_memory=True) if "spill_" in args.workload else None
    cap = min(n, d)
    outs = isa._alloc_outputs(torch, cap, aggs, "cuda")
    out = isa._output_struct(outs, cap)
    inp = isa.isa_input(isa._ptr(kd), isa._ptr(vd), isa._ptr(fd), n)
    wss = isa.isa_workspace(isa._ptr(ws), budget)
    sps = isa.isa_spill(isa._ptr(spill), spill.numel() if spill is not None else 0)
    st = isa.isa_stats()
    stream = torch.cuda.current_stream()
    sp = isa._stream_ptr(stream)

    def step():
        rc = L.isa_group_by(ctx.handle, isa.ctypes.byref(inp), aggs, wss, sps, isa.ctypes.byref(out),
                            isa.ctypes.byref(st), sp)
        if rc != isa.ISA_OK:
            raise isa.InsortError(rc, ctx.last_error())

    for i in range(args.warmup):
        step()
        print("bench: warmup %d done" % i, file=sys.stderr, flush=True)
    if not args.no_profile:
        ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        print("bench: step %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = ctx.profile_read() if not args.no_profile else {}
    ctx.profile(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    groups = out.n_groups
    stats = st.as_dict()

    in_row = 8 + (8 if aggs & (isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64) else 0) + (8 if with_f else 0)
    algo_bytes = n * in_row + groups * row_b
    step_gbs = algo_bytes / (ms_per_step * 1e-3) / 1e9

    roofline = None
    kernels = {}
    if prof:
        for name, r in prof.items():
            kernels[name] = {"launches": r["launches"], "avg_us": 1e3 * r["total_ms"] / max(1, r["launches"]),
                             "ms_per_step": r["total_ms"] / args.steps,
                             "rows_per_launch": r["rows"] / max(1, r["launches"]),
                             "algo_GBps": (r["bytes"] / (r["total_ms"] * 1e-3) / 1e9) if r["total_ms"] else None}
        dev_kernels = {k: v for k, v in prof.items() if k.startswith("k_")}
        dom = max(dev_kernels, key=lambda k: dev_kernels[k]["total_ms"])
        r = dev_kernels[dom]
        achieved = r["bytes"] / (r["total_ms"] * 1e-3) / 1e9
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                    "avg_launch_us": round(1e3 * r["total_ms"] / r["launches"], 2),
                    "algo_bytes_per_launch": int(r["bytes"] / r["launches"])}

    host_link = None
    if stats["spilled_rows"]:
        hb = 2 * stats["spilled_bytes"]
        hl_ms = sum(prof[k]["total_ms"] for k in ("spill_d2h", "merge_h2d") if k in prof) / args.steps
        host_link = {"bytes_per_step": hb, "copy_ms_per_step": round(hl_ms, 2),
                     "GBps": round(hb / (hl_ms * 1e-3) / 1e9, 1) if hl_ms else None}

    cpu = None
    if args.cpu_sample:
        import oracle
        m = min(args.cpu_sample, n)
        k_h = kd[:m].cpu().numpy().view(np.uint64)
        v_h = vd[:m].cpu().numpy()
        f_h = fd[:m].cpu().numpy() if fd is not None else None
        print("bench: timing the CPU oracle on %d rows" % m, file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        oracle.group_by(k_h, v_h, f_h)
        c1 = time.perf_counter()
        cpu = {"value": round(m / (c1 - c0), 1), "unit": "rows/s", "cores": 1, "kind": "oracle",
               "sample": "first %d rows of the same input, single-threaded C oracle "
                         "(merge sort then in-stream aggregation)" % m}

    res = {
        "metric": "input rows/s aggregated (% HBM roofline)",
        "value": round(n / (ms_per_step * 1e-3), 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64+i64+f64" if with_f else "u64+i64",
        "data": "synthetic",
        "config": {"workload": args.workload, "rows": n, "distinct_domain": d, "zipf_s": s,
                   "budget_bytes": budget, "aggs": aggs_name, "groups": groups},
        "hbm_algo_GBps_whole_step": round(step_gbs, 1),
        "hbm_roofline_frac_whole_step": round(step_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_link": host_link,
        "stats": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()},
        "kernels": kernels,
    }
    print(json.dumps(res))
    ctx.close()


if __name__ == "__main__":
    main()

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
LINK_PEAK_GBS = 64.0   # host link: PCIe 5.0 x16, published rate per direction

WORKLOADS = {
    # name: (rows, distinct domain, zipf s, seed, budget MiB, with f64, aggs name)
    "spill_100M_zipf0.8": (100_000_000, 10_000_000, 0.8, 3, 256, True, "all"),
    "spill_100M_zipf0": (100_000_000, 10_000_000, 0.0, 2, 256, True, "all"),
    "spill_100M_zipf1.2": (100_000_000, 10_000_000, 1.2, 4, 256, True, "all"),
    # the same inputs with run generation by replacement selection through the index
    "spill_100M_zipf0.8_rs": (100_000_000, 10_000_000, 0.8, 3, 256, True, "all"),
    "spill_100M_zipf0_rs": (100_000_000, 10_000_000, 0.0, 2, 256, True, "all"),
    "nospill_100M_zipf0.8": (100_000_000, 10_000_000, 0.8, 3, 12 * 1024, True, "all"),
    "nospill_100M_zipf0": (100_000_000, 10_000_000, 0.0, 2, 12 * 1024, True, "all"),
    "nospill_100M_zipf1.2": (100_000_000, 10_000_000, 1.2, 4, 12 * 1024, True, "all"),
    "plain_1M_10k": (1_000_000, 10_000, 0.0, 1, 64, False, "int"),
    # input already sorted on the key (in-stream aggregation, no sort): keys are
    # 1e8 ranks uniform over 1e7 values, sorted on the device
    "sorted_100M_1e7": (100_000_000, 10_000_000, 0.0, 8, 16, True, "all"),
    # count(*) + count(distinct x) group by g: int32 g uniform over 1e3 values,
    # int32 x uniform over 1e4 values (about 1e7 distinct pairs), 256 MiB workspace
    "cdistinct_100M": (100_000_000, 10_000_000, 0.0, 9, 256, False, "count"),
}
# Forms beyond the plain operator (each prints its own JSON line):
#   batch_c3:    instances with rows log-uniform 1e3..1e7 and distinct/rows
#                log-uniform 1e-4..1, uint64 key, int64 value (count of
#                instances from --instances); batched launch vs per-instance calls
#   batch_small: the same with rows log-uniform 1e3..1e5 (launch-bound regime)
#   serve_c4:    Poisson stream of requests, rows log-uniform 1e4..1e8, distinct
#                ratio log-uniform 1e-4..1, Zipf s uniform in [0, 1.2]; server
#                (continuous batching, 64 GiB workspace cap) vs FIFO plain calls
FORMS = ("batch_c3", "batch_small", "serve_c4")


def _instances(seed, count, lo, hi):
    import numpy as np
    rng = np.random.default_rng(seed)
    rows = np.exp(rng.uniform(np.log(lo), np.log(hi), count)).round().astype(np.int64)
    ratio = np.exp(rng.uniform(np.log(1e-4), 0.0, count))
    d = np.maximum(1, np.round(rows * ratio)).astype(np.int64)
    return rows, d, rng


def bench_batch(args, lo, hi):
    import ctypes
    import numpy as np
    import torch

    import datagen
    import datagen.device as dgd
    import paper_2010_00152_amd as isa

    count = args.instances
    rows, d, _ = _instances(6, count, lo, hi)
    ctx = isa.Context(0)
    L = isa.lib()
    aggs = isa.ISA_INT_AGGS
    wave_rows = 200_000_000
    ws = torch.empty(24 << 30, dtype=torch.uint8, device="cuda")
    wss = isa.isa_workspace(isa._ptr(ws), ws.numel())
    sp = isa._stream_ptr()
    t_batch = t_graphless = t_plain = 0.0
    total_rows = int(rows.sum())
    i0 = 0
    waves = 0
    # launch configuration: from the tuning table if it holds this workload's
    # signature, else autotuned on the first wave (untimed) and recorded
    from paper_2010_00152_amd.tuning import TuningTable, signature
    table = TuningTable(args.tuning_file)
    sig = signature(rows, aggs)
    tuned = table.lookup(sig)
    tune_info = {"source": "table" if tuned else "autotuned on the first wave"}
    if tuned:
        ctx.set_tuning(**tuned)
    while i0 < count:
        i1, acc = i0, 0
        while i1 < count and (acc + rows[i1] <= wave_rows or i1 == i0):
            acc += int(rows[i1])
            i1 += 1
        n_w = i1 - i0
        keys = torch.empty(acc, dtype=torch.int64, device="cuda")
        vals = torch.empty(acc, dtype=torch.int64, device="cuda")
        outs_mem = [torch.empty(acc, dtype=torch.int64, device="cuda") for _ in range(5)]
        ins = (isa.isa_input * n_w)()
        outs = (isa.isa_output * n_w)()
        off = 0
        for j, i in enumerate(range(i0, i1)):
            n = int(rows[i])
            seed = datagen.substream_seed(6, i)
            dgd.keys(datagen.substream_seed(seed, 1), n, int(d[i]), 0.0, out=keys[off:off + n])
            dgd.uniform_i64(datagen.substream_seed(seed, 2), n, out=vals[off:off + n])
            ins[j] = isa.isa_input(keys[off:].data_ptr(), vals[off:].data_ptr(), None, n)
            outs[j] = isa.isa_output(outs_mem[0][off:].data_ptr(), outs_mem[1][off:].data_ptr(),
                                     outs_mem[2][off:].data_ptr(), None, outs_mem[3][off:].data_ptr(),
                                     outs_mem[4][off:].data_ptr(), n, 0)
            off += n
        torch.cuda.synchronize()

        def batched():
            rc = L.isa_batch_run(ctx.handle, n_w, ins, aggs, wss, outs, sp)
            if rc != isa.ISA_OK:
                raise isa.InsortError(rc, ctx.last_error())

        if tuned is None:
            nc = L.isa_tune_candidates(None, 0)
            times = (isa.ctypes.c_double * nc)()
            best = isa.isa_tuning()
            rc = L.isa_tune_batch(ctx.handle, n_w, ins, aggs, wss, outs, sp, isa.ctypes.byref(best), times, nc)
            if rc != isa.ISA_OK:
                raise isa.InsortError(rc, ctx.last_error())
            tuned = best.as_dict()
            cands = isa.tune_candidates()
            dflt = cands.index(isa.Context.default_tuning())
            tune_info.update({"first_wave_ms_default": round(times[dflt], 3),
                              "first_wave_ms_tuned": round(min(times[i] for i in range(nc)), 3),
                              "candidates": nc})
            table.record(sig, tuned, min(times[i] for i in range(nc)))
            print("bench: tuned %s" % tuned, file=sys.stderr, flush=True)
        batched()  # warm
        ctx.set_tuning(**tuned)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        batched()
        torch.cuda.synchronize()
        t_batch += time.perf_counter() - t0
        ctx.set_tuning()  # the library's default configuration
        t0 = time.perf_counter()
        batched()
        torch.cuda.synchronize()
        t_graphless += time.perf_counter() - t0
        ctx.set_tuning(**tuned)
        sps = isa.isa_spill(None, 0)
        t0 = time.perf_counter()
        for j in range(n_w):
            rc = L.isa_group_by(ctx.handle, ctypes.byref(ins[j]), aggs, wss, sps, ctypes.byref(outs[j]), None, sp)
            if rc != isa.ISA_OK:
                raise isa.InsortError(rc, ctx.last_error())
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t0
        waves += 1
        print("bench: wave %d (%d instances, %d rows) done" % (waves, n_w, acc), file=sys.stderr, flush=True)
        del keys, vals, outs_mem
        i0 = i1
    res = {
        "metric": "input rows/s aggregated, batched launch vs per-instance plain calls",
        "value": round(total_rows / t_batch, 1),
        "unit": "rows/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "data": "synthetic",
        "dtype": "u64+i64",
        "config": {"workload": args.workload, "instances": count, "rows_lo": lo, "rows_hi": hi,
                   "total_rows": total_rows, "waves": waves},
        "batched_tuned_rows_per_s": round(total_rows / t_batch, 1),
        "batched_default_config_rows_per_s": round(total_rows / t_graphless, 1),
        "plain_per_instance_rows_per_s": round(total_rows / t_plain, 1),
        "speedup_vs_plain": round(t_plain / t_batch, 3),
        "tuning": dict(tuned, **tune_info),
        "ms": {"batched_tuned": round(1e3 * t_batch, 2), "batched_default_config": round(1e3 * t_graphless, 2),
               "plain": round(1e3 * t_plain, 2)},
    }
    print(json.dumps(res))
    ctx.close()


def bench_serve(args):
    import ctypes
    import numpy as np
    import torch

    import datagen
    import datagen.device as dgd
    import paper_2010_00152_amd as isa

    n_req = args.requests
    rows, d, rng = _instances(7, n_req, 1e4, 1e8)
    s_zipf = rng.uniform(0.0, 1.2, n_req)
    ctx = isa.Context(0)
    L = isa.lib()
    aggs = isa.ISA_INT_AGGS
    cap = 64 << 30
    ws_srv = torch.empty(cap, dtype=torch.uint8, device="cuda")
    gen_stream = torch.cuda.Stream()

    def make(i):
        n = int(rows[i])
        seed = datagen.substream_seed(7, i)
        with torch.cuda.stream(gen_stream):
            k = dgd.zipf_approx_keys(datagen.substream_seed(seed, 1), n, int(d[i]), float(s_zipf[i]))
            v = dgd.uniform_i64(datagen.substream_seed(seed, 2), n)
        gen_stream.synchronize()
        return k, v

    # the plain rate of this GPU sets the arrival rate (rho * R_plain / E[rows])
    sp = isa._stream_ptr()
    wsp = isa.isa_workspace(isa._ptr(ws_srv), cap)
    nosp = isa.isa_spill(None, 0)

    def plain(k, v):
        n = k.numel()
        o = isa._alloc_outputs(torch, n, aggs, "cuda")
        out = isa._output_struct(o, n)
        inp = isa.isa_input(k.data_ptr(), v.data_ptr(), None, n)
        rc = L.isa_group_by(ctx.handle, ctypes.byref(inp), aggs, wsp, nosp, ctypes.byref(out), None, sp)
        if rc != isa.ISA_OK:
            raise isa.InsortError(rc, ctx.last_error())
        torch.cuda.synchronize()
        return out.n_groups

    k, v = make(0)
    plain(k, v)
    # R_plain: plain-path rate on the first requests of the trace (group-by time only)
    tt, cal_rows = 0.0, 0
    for i in range(min(8, n_req)):
        k, v = make(i)
        t1 = time.perf_counter()
        plain(k, v)
        tt += time.perf_counter() - t1
        cal_rows += int(rows[i])
    del k, v
    r_plain = cal_rows / tt
    lam = args.rho * r_plain / float(rows.mean())
    arrivals = np.cumsum(rng.exponential(1.0 / lam, n_req))
    print("bench: plain %.3g rows/s, arrival rate %.1f req/s over %.1f s" % (r_plain, lam, arrivals[-1]),
          file=sys.stderr, flush=True)

    def run(mode):
        # latency = scheduled arrival -> output ready; a request the client
        # reaches late (the previous plain call still running) waits from its
        # scheduled arrival, as in a FIFO queue
        lat = np.zeros(n_req)
        srv = isa.Server(ctx, cap, slots=args.slots, workspace=ws_srv) if mode == "server" else None
        pending = {}
        start = time.perf_counter()
        for i in range(n_req):
            now = time.perf_counter() - start
            if arrivals[i] > now:
                time.sleep(arrivals[i] - now)
            k, v = make(i)
            if mode == "server":
                late_ms = 1e3 * (time.perf_counter() - start - arrivals[i])
                t = srv.submit(k, v, None, aggs=aggs)
                pending[t] = (i, late_ms)
                for tk in list(pending):
                    done, lat_ms, st = srv.poll(tk)
                    if done:
                        if st != isa.ISA_OK:
                            raise isa.InsortError(st, "request %d" % pending[tk][0])
                        j, late = pending.pop(tk)
                        lat[j] = lat_ms + late
                        srv.live.pop(tk, None)
            else:
                plain(k, v)
                lat[i] = 1e3 * (time.perf_counter() - start - arrivals[i])
            del k, v
            if i % 200 == 0:
                print("bench: %s request %d" % (mode, i), file=sys.stderr, flush=True)
        if srv is not None:
            srv.drain()
            for tk in list(pending):
                done, lat_ms, st = srv.poll(tk)
                if st != isa.ISA_OK:
                    raise isa.InsortError(st, "request %d" % pending[tk][0])
                j, late = pending.pop(tk)
                lat[j] = lat_ms + late
            srv.close()
        wall = time.perf_counter() - start
        return lat, wall

    lat_s, wall_s = run("server")
    lat_f, wall_f = run("fifo")
    tot = int(rows.sum())
    res = {
        "metric": "p50/p99 latency batched vs plain; input rows/s aggregated",
        "value": round(float(np.percentile(lat_s, 99)), 3),
        "unit": "ms (p99, server)",
        "n_gpus": 1,
        "higher_is_better": False,
        "data": "synthetic",
        "dtype": "u64+i64",
        "config": {"workload": "serve_c4", "requests": n_req, "rho": args.rho, "slots": args.slots,
                   "hbm_cap_bytes": cap, "total_rows": tot},
        "server": {"p50_ms": round(float(np.percentile(lat_s, 50)), 3),
                   "p99_ms": round(float(np.percentile(lat_s, 99)), 3),
                   "rows_per_s": round(tot / wall_s, 1), "wall_s": round(wall_s, 3)},
        "fifo_plain": {"p50_ms": round(float(np.percentile(lat_f, 50)), 3),
                       "p99_ms": round(float(np.percentile(lat_f, 99)), 3),
                       "rows_per_s": round(tot / wall_f, 1), "wall_s": round(wall_f, 3)},
        "plain_rate_rows_per_s": round(r_plain, 1),
    }
    print(json.dumps(res))
    ctx.close()


# Profile labels of the library's launches -> kernel names in rocprofv3 output
KERNELS_OF_LABEL = {"k_leaf": ["k_leaf_flat", "k_leaf"], "k_merge": ["k_merge"], "k_scatter": ["k_scatter"],
                    "k_hist": ["k_hist"], "k_sample": ["k_sample", "k_sample_keys"]}


def link_summary(spilled_bytes, link_ms, ms_per_step):
    """Host-link figures of a spilling step: runs go out during run generation
    and come back during the wide merge, which starts only once every run is
    written, so the step's link floor is both volumes at the link's peak."""
    hb = 2 * spilled_bytes
    gbs = hb / (link_ms * 1e-3) / 1e9 if link_ms else None
    floor_ms = hb / (LINK_PEAK_GBS * 1e9) * 1e3
    return {"bytes_per_step": hb, "copy_ms_per_step": round(link_ms, 2),
            "GBps": round(gbs, 1) if gbs else None, "peak_GBps": LINK_PEAK_GBS,
            "frac": round(gbs / LINK_PEAK_GBS, 3) if gbs else None,
            "floor_ms_per_step": round(floor_ms, 2),
            "step_frac_of_floor": round(floor_ms / ms_per_step, 3) if ms_per_step else None}


def hbm_traffic(workload, label):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated) of the kernels
    behind a profile label, from profiles/hbm_traffic.json; None when the
    workload was not profiled or the kernels changed since (source hash)."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", "hbm_traffic.json")) as f:
            t = json.load(f)
        src = open(os.path.join(here, "paper_2010_00152_amd", "csrc", "isa_kernels.hip"), "rb").read()
    except OSError:
        return None, None
    if hashlib.sha256(src).hexdigest()[:16] != t.get("kernel_source_sha256_16"):
        return None, None
    wl = t.get("workloads", {}).get(workload)
    if not wl:
        return None, None
    n = b = 0.0
    for k in KERNELS_OF_LABEL.get(label, [label]):
        if k in wl:
            n += wl[k]["launches"]
            b += wl[k]["launches"] * (wl[k]["fetch_bytes_per_launch"] + wl[k]["write_bytes_per_launch"])
    return (b / n, None) if n else (None, None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="spill_100M_zipf0.8", choices=sorted(WORKLOADS) + list(FORMS))
    ap.add_argument("--instances", type=int, default=10000, help="batch_*: number of instances")
    ap.add_argument("--requests", type=int, default=2000, help="serve_c4: number of requests")
    ap.add_argument("--rho", type=float, default=0.8, help="serve_c4: offered load vs the plain rate")
    ap.add_argument("--slots", type=int, default=3, help="serve_c4: concurrent server batches")
    ap.add_argument("--tuning-file", default=None,
                    help="batch_*: JSON table of autotuned launch configurations (read, and written when tuning)")
    ap.add_argument("--cpu-sample", type=int, default=10_000_000,
                    help="rows of the input the CPU oracle is timed on (0 = skip)")
    ap.add_argument("--no-profile", action="store_true", help="skip per-kernel event timing")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="extra untimed steps with per-kernel HIP-event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (--gpus %d requested); "
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

    if args.workload == "batch_c3":
        return bench_batch(args, 1e3, 1e7)
    if args.workload == "batch_small":
        return bench_batch(args, 1e3, 1e5)
    if args.workload == "serve_c4":
        return bench_serve(args)

    import datagen
    import datagen.device as dgd
    import paper_2010_00152_amd as isa

    n, d, s, seed, budget_mib, with_f, aggs_name = WORKLOADS[args.workload]
    aggs = {"all": isa.ISA_ALL, "int": isa.ISA_INT_AGGS, "count": isa.ISA_COUNT}[aggs_name]
    print("bench: workload %s, generating %d rows on the device" % (args.workload, n), file=sys.stderr,
          flush=True)
    if args.workload.startswith("cdistinct_"):
        gd = dgd.uniform_ranks(datagen.substream_seed(seed, 1), n, 1000).to(torch.int32)
        xd = dgd.uniform_ranks(datagen.substream_seed(seed, 2), n, 10_000).to(torch.int32)
        kd, vd, fd = gd, None, None
        cd_scratch = torch.empty(24 * n, dtype=torch.uint8, device="cuda")
        cd_out = [torch.empty(1000, dtype=t, device="cuda") for t in (torch.int32, torch.int64, torch.int64)]
        cd_n = isa.ctypes.c_uint64()
    elif args.workload.startswith("sorted_"):
        kd = torch.sort(dgd.uniform_ranks(datagen.substream_seed(seed, 1), n, d)).values
        vd = dgd.uniform_i64(datagen.substream_seed(seed, 2), n)
        fd = dgd.normal_f64(datagen.substream_seed(seed, 3), n) if with_f else None
    else:
        kd, vd, fd = dgd.plain_input(seed, n, d, s, with_f64=with_f)
    torch.cuda.synchronize()
    ctx = isa.Context(0)
    if args.workload.endswith("_rs"):
        ctx.set_run_generation(isa.ISA_RUNGEN_REPLACEMENT)
    L = isa.lib()
    budget = budget_mib << 20
    ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
    row_b = L.isa_state_row_bytes(aggs)
    spilling = "spill_" in args.workload or args.workload.startswith("cdistinct_")
    spill = torch.empty(n * row_b, dtype=torch.uint8, pin_memory=True) if spilling else None
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
        if args.workload.startswith("cdistinct_"):
            rc = L.isa_count_distinct(ctx.handle, isa._ptr(gd), isa._ptr(xd), n, wss, sps, isa._ptr(cd_scratch),
                                      cd_scratch.numel(), isa._ptr(cd_out[0]), isa._ptr(cd_out[1]),
                                      isa._ptr(cd_out[2]), 1000, isa.ctypes.byref(cd_n), sp)
            out.n_groups = cd_n.value
        elif args.workload.startswith("sorted_"):
            rc = L.isa_group_by_sorted(ctx.handle, isa.ctypes.byref(inp), aggs, wss, isa.ctypes.byref(out), sp)
        else:
            rc = L.isa_group_by(ctx.handle, isa.ctypes.byref(inp), aggs, wss, sps, isa.ctypes.byref(out),
                                isa.ctypes.byref(st), sp)
        if rc != isa.ISA_OK:
            raise isa.InsortError(rc, ctx.last_error())

    for i in range(args.warmup):
        step()
        print("bench: warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        step()
        print("bench: step %d done (%.1f ms host)" % (i, (time.perf_counter() - ts) * 1e3), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    # phase times of the last timed call (the profiled calls below add event records)
    timed_phases = {k: round(v, 3) for k, v in st.as_dict().items() if k.startswith("t_")}
    # per-kernel HIP-event timing in separate steps, so that the event records
    # do not enter the timed steps above
    prof = {}
    prof_steps = 0 if args.no_profile else args.profile_steps
    if prof_steps:
        ctx.profile(True)
        for i in range(prof_steps):
            step()
        torch.cuda.synchronize()
        prof = ctx.profile_read()
        ctx.profile(False)
        print("bench: %d profiled step(s) done" % prof_steps, file=sys.stderr, flush=True)
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
                             "ms_per_step": r["total_ms"] / prof_steps,
                             "rows_per_launch": r["rows"] / max(1, r["launches"]),
                             "algo_GBps": (r["bytes"] / (r["total_ms"] * 1e-3) / 1e9) if r["total_ms"] else None}
        dev_kernels = {k: v for k, v in prof.items() if k.startswith("k_")}
        dom = max(dev_kernels, key=lambda k: dev_kernels[k]["total_ms"])
        r = dev_kernels[dom]
        achieved = r["bytes"] / (r["total_ms"] * 1e-3) / 1e9
        algo_pl = r["bytes"] / r["launches"]
        traffic, ratio = hbm_traffic(args.workload, dom)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                    "traffic": int(traffic) if traffic else None,
                    "traffic_over_algo": round(traffic / algo_pl, 3) if traffic else None,
                    "avg_launch_us": round(1e3 * r["total_ms"] / r["launches"], 2),
                    "algo_bytes_per_launch": int(algo_pl)}

    host_link = None
    if stats["spilled_rows"]:
        hl_ms = sum(prof[k]["total_ms"] for k in ("spill_d2h", "merge_h2d") if k in prof) / max(1, prof_steps)
        host_link = link_summary(stats["spilled_bytes"], hl_ms, ms_per_step)

    cpu = None
    if args.cpu_sample:
        import oracle
        m = min(args.cpu_sample, n)
        print("bench: timing the CPU oracle on %d rows" % m, file=sys.stderr, flush=True)
        if args.workload.startswith("cdistinct_"):
            g_h = gd[:m].cpu().numpy().astype(np.uint64)
            x_h = xd[:m].cpu().numpy().astype(np.uint64)
            c0 = time.perf_counter()
            oracle.count_distinct(g_h, x_h)
            c1 = time.perf_counter()
        else:
            k_h = kd[:m].cpu().numpy().view(np.uint64)
            v_h = vd[:m].cpu().numpy()
            f_h = fd[:m].cpu().numpy() if fd is not None else None
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
                   "budget_bytes": budget, "aggs": aggs_name, "groups": groups,
                   "run_generation": "replacement" if args.workload.endswith("_rs") else "read-sort-write"},
        "hbm_algo_GBps_whole_step": round(step_gbs, 1),
        "hbm_roofline_frac_whole_step": round(step_gbs / HBM_PEAK_GBS, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "host_link": host_link,
        "stats": {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()},
        "phases_timed_ms": timed_phases,
        "kernels": kernels,
    }
    print(json.dumps(res))
    ctx.close()


if __name__ == "__main__":
    main()

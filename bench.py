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
    # (A, B) int32 pairs, 1e3 A values sorted, 1e5 B values per A, int64 value,
    # grouped one A-segment at a time (rows, -, -, seed, budget MiB, -, aggs)
    "segmented_200M": (200_000_000, 0, 0.0, 5, 256, False, "int"),
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
    tune_info = {"source": "table" if tuned else "autotuned on a sample of the whole workload"}
    if tuned:
        ctx.set_tuning(**tuned)
    else:
        # an unbiased sample of the whole workload: every instance at a fixed
        # stride (sizes are drawn independently per instance), about 2e8 rows
        stride = max(1, int(np.ceil(float(rows.sum()) / 2e8)))
        pick = list(range(0, count, stride))
        acc = int(rows[pick].sum())
        n_s = len(pick)
        keys_s = torch.empty(acc, dtype=torch.int64, device="cuda")
        vals_s = torch.empty(acc, dtype=torch.int64, device="cuda")
        outs_s = [torch.empty(acc, dtype=torch.int64, device="cuda") for _ in range(5)]
        ins_s = (isa.isa_input * n_s)()
        outs_st = (isa.isa_output * n_s)()
        off = 0
        for j, i in enumerate(pick):
            n = int(rows[i])
            seed = datagen.substream_seed(6, i)
            dgd.keys(datagen.substream_seed(seed, 1), n, int(d[i]), 0.0, out=keys_s[off:off + n])
            dgd.uniform_i64(datagen.substream_seed(seed, 2), n, out=vals_s[off:off + n])
            ins_s[j] = isa.isa_input(keys_s[off:].data_ptr(), vals_s[off:].data_ptr(), None, n)
            outs_st[j] = isa.isa_output(outs_s[0][off:].data_ptr(), outs_s[1][off:].data_ptr(),
                                        outs_s[2][off:].data_ptr(), None, outs_s[3][off:].data_ptr(),
                                        outs_s[4][off:].data_ptr(), n, 0)
            off += n
        torch.cuda.synchronize()
        nc = L.isa_tune_candidates(None, 0)
        times = (isa.ctypes.c_double * nc)()
        best = isa.isa_tuning()
        rc = L.isa_tune_batch(ctx.handle, n_s, ins_s, aggs, wss, outs_st, sp, isa.ctypes.byref(best), times, nc)
        if rc != isa.ISA_OK:
            raise isa.InsortError(rc, ctx.last_error())
        tuned = best.as_dict()
        cands = isa.tune_candidates()
        dflt = cands.index(isa.Context.default_tuning())
        tune_info.update({"sample_instances": n_s, "sample_rows": acc,
                          "sample_ms_default": round(times[dflt], 3),
                          "sample_ms_tuned": round(min(times[i] for i in range(nc)), 3), "candidates": nc})
        table.record(sig, tuned, min(times[i] for i in range(nc)))
        print("bench: tuned %s on %d sampled instances" % (tuned, n_s), file=sys.stderr, flush=True)
        del keys_s, vals_s, outs_s
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
    ctx.close()
    return res


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
                        srv.release(tk)
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
    ctx.close()
    return res


# Profile labels of the library's launches -> kernel names in rocprofv3 output
KERNELS_OF_LABEL = {"k_leaf": ["k_leaf_flat", "k_leaf"], "k_merge": ["k_merge"], "k_scatter": ["k_scatter"],
                    "k_hist": ["k_hist", "k_hist_batch"], "k_sample": ["k_sample", "k_sample_keys"],
                    "merge_h2d": ["k_gather"]}
# input generators: not part of a step, left out of the step's counter bytes
GENERATORS = ("k_zipf_keys", "k_normal_f64", "k_uniform_i64", "k_uniform_ranks", "k_keys_uniform",
              "k_seg_", "k_zipf_approx")


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


def _profiles(name):
    """A committed profile table (profiles/<name>) if it was taken on the
    current kernel source (same sha256 prefix), else None."""
    import hashlib
    here = os.path.dirname(os.path.abspath(__file__))
    try:
        with open(os.path.join(here, "profiles", name)) as f:
            t = json.load(f)
        src = open(os.path.join(here, "paper_2010_00152_amd", "csrc", "isa_kernels.hip"), "rb").read()
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest()[:16] != t.get("kernel_source_sha256_16"):
        return None
    return t


def step_traffic(workload):
    """HBM bytes of one step from rocprofv3 FETCH_SIZE and WRITE_SIZE
    (copy-calibrated), summed over the step's kernels; None when the workload
    was not profiled on the current kernel source."""
    t = _profiles("hbm_traffic.json")
    wl = (t or {}).get("workloads", {}).get(workload)
    if not wl:
        return None
    return sum(r["launches"] * (r["fetch_bytes_per_launch"] + r["write_bytes_per_launch"])
               for k, r in wl.items() if not k.startswith(GENERATORS)) / max(1, t.get("steps", {}).get(workload, 1))


def rocprof_dominant(workload):
    """(kernel, avg us, launches per step) of the kernel with the most time in
    the committed rocprofv3 summary of this workload, or None."""
    t = _profiles("kernel_stats.json")
    wl = (t or {}).get("workloads", {}).get(workload)
    if not wl:
        return None
    ks = {k: r for k, r in wl["kernels"].items() if not k.startswith(GENERATORS) and not k.startswith("__")}
    k = max(ks, key=lambda x: ks[x]["total_us"])
    return k, ks[k]["avg_us"], ks[k]["calls"] / max(1, wl.get("calls", 1))


def host_info():
    import platform
    model = platform.processor() or ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram = round(int(line.split()[1]) / 2**20, 1)
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "nproc_online": os.cpu_count(), "cpus_usable": usable, "ram_GiB": ram}


# host threads given to the parallel oracle: the CPU share of a one-GPU machine
ORACLE_THREADS = 16


def cpu_oracle(kd, vd, fd, n, sample_rows, parallel):
    """The C oracle on this host: single-threaded on the first sample_rows rows
    (a bounded sample), and, with `parallel`, its multi-threaded form (the same
    sort-then-scan over sampled key ranges) on the whole input."""
    import numpy as np
    import oracle
    m = min(sample_rows, n)
    print("bench: timing the CPU oracle on %d rows (1 thread)" % m, file=sys.stderr, flush=True)
    k_h = kd.cpu().numpy().view(np.uint64)
    v_h = vd.cpu().numpy() if vd is not None else None
    f_h = fd.cpu().numpy() if fd is not None else None
    c0 = time.perf_counter()
    oracle.group_by(k_h[:m], None if v_h is None else v_h[:m], None if f_h is None else f_h[:m])
    c1 = time.perf_counter()
    one = {"value": round(m / (c1 - c0), 1), "unit": "rows/s", "cores": 1, "kind": "oracle",
           "sample": "first %d rows of the same input, single-threaded C oracle "
                     "(merge sort then in-stream aggregation), %.1f s" % (m, c1 - c0)}
    par = None
    if parallel:
        threads = min(ORACLE_THREADS, oracle.nproc())
        print("bench: timing the CPU oracle on %d rows (%d threads)" % (n, threads), file=sys.stderr, flush=True)
        c0 = time.perf_counter()
        oracle.group_by(k_h, v_h, f_h, threads=threads)
        c1 = time.perf_counter()
        par = {"value": round(n / (c1 - c0), 1), "unit": "rows/s", "cores": threads, "kind": "oracle",
               "sample": "the whole input (%d rows), the C oracle's sort-then-scan over sampled key ranges on "
                         "%d host threads, %.1f s" % (n, threads, c1 - c0)}
    return one, par


def make_input(torch, dgd, datagen, workload):
    n, d, s, seed, budget_mib, with_f, aggs_name = WORKLOADS[workload]
    if workload.startswith("cdistinct_"):
        gd = dgd.uniform_ranks(datagen.substream_seed(seed, 1), n, 1000).to(torch.int32)
        xd = dgd.uniform_ranks(datagen.substream_seed(seed, 2), n, 10_000).to(torch.int32)
        return gd, xd, None
    if workload.startswith("segmented_"):
        return dgd.segmented_input(seed, n)
    if workload.startswith("sorted_"):
        kd = torch.sort(dgd.uniform_ranks(datagen.substream_seed(seed, 1), n, d)).values
        vd = dgd.uniform_i64(datagen.substream_seed(seed, 2), n)
        fd = dgd.normal_f64(datagen.substream_seed(seed, 3), n) if with_f else None
        return kd, vd, fd
    return dgd.plain_input(seed, n, d, s, with_f64=with_f)


def run_workload(args, workload, steps, warmup, detail):
    """Time `steps` whole calls of one workload (inputs resident in HBM) and
    return its figures; with `detail`, also the per-kernel event timing, the
    dominant kernel and the CPU oracle."""
    import numpy as np
    import torch

    import datagen
    import datagen.device as dgd
    import paper_2010_00152_amd as isa

    n, d, s, seed, budget_mib, with_f, aggs_name = WORKLOADS[workload]
    aggs = {"all": isa.ISA_ALL, "int": isa.ISA_INT_AGGS, "count": isa.ISA_COUNT}[aggs_name]
    print("bench: workload %s, generating %d rows on the device" % (workload, n), file=sys.stderr, flush=True)
    a0, a1, a2 = make_input(torch, dgd, datagen, workload)
    torch.cuda.synchronize()
    ctx = isa.Context(0)
    if workload.endswith("_rs"):
        ctx.set_run_generation(isa.ISA_RUNGEN_REPLACEMENT)
    L = isa.lib()
    budget = budget_mib << 20
    ws = torch.empty(budget, dtype=torch.uint8, device="cuda")
    wss = isa.isa_workspace(isa._ptr(ws), budget)
    row_b = L.isa_state_row_bytes(aggs)
    spilling = "spill_" in workload or workload.startswith("cdistinct_")
    spill = torch.empty(n * row_b, dtype=torch.uint8, pin_memory=True) if spilling else None
    sps = isa.isa_spill(isa._ptr(spill), spill.numel() if spill is not None else 0)
    st = isa.isa_stats()
    stream = torch.cuda.current_stream()
    sp = isa._stream_ptr(stream)
    segmented = workload.startswith("segmented_")
    cap = n if segmented else min(n, d)
    outs = isa._alloc_outputs(torch, cap, aggs, "cuda", with_keys=not segmented)
    out = isa._output_struct(outs, cap)
    if segmented:
        seg_a = torch.empty(cap, dtype=torch.int32, device="cuda")
        seg_b = torch.empty(cap, dtype=torch.int32, device="cuda")
    if workload.startswith("cdistinct_"):
        cd_scratch = torch.empty(24 * n, dtype=torch.uint8, device="cuda")
        cd_out = [torch.empty(1000, dtype=t, device="cuda") for t in (torch.int32, torch.int64, torch.int64)]
        cd_n = isa.ctypes.c_uint64()
    inp = isa.isa_input(isa._ptr(a0), isa._ptr(a1), isa._ptr(a2), n)

    def step():
        if workload.startswith("cdistinct_"):
            rc = L.isa_count_distinct(ctx.handle, isa._ptr(a0), isa._ptr(a1), n, wss, sps, isa._ptr(cd_scratch),
                                      cd_scratch.numel(), isa._ptr(cd_out[0]), isa._ptr(cd_out[1]),
                                      isa._ptr(cd_out[2]), 1000, isa.ctypes.byref(cd_n), sp)
            out.n_groups = cd_n.value
        elif workload.startswith("sorted_"):
            rc = L.isa_group_by_sorted(ctx.handle, isa.ctypes.byref(inp), aggs, wss, isa.ctypes.byref(out), sp)
        elif segmented:
            rc = L.isa_group_by_segmented(ctx.handle, isa._ptr(a0), isa._ptr(a1), isa._ptr(a2), n, aggs, wss,
                                          isa._ptr(seg_a), isa._ptr(seg_b), isa.ctypes.byref(out), sp)
        else:
            rc = L.isa_group_by(ctx.handle, isa.ctypes.byref(inp), aggs, wss, sps, isa.ctypes.byref(out),
                                isa.ctypes.byref(st), sp)
        if rc != isa.ISA_OK:
            raise isa.InsortError(rc, ctx.last_error())

    for i in range(warmup):
        step()
        print("bench: %s warmup %d done" % (workload, i), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ts = time.perf_counter()
        step()
        print("bench: %s step %d done (%.1f ms host)" % (workload, i, (time.perf_counter() - ts) * 1e3),
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / steps
    timed_phases = {k: round(v, 3) for k, v in st.as_dict().items() if k.startswith("t_")}
    groups = out.n_groups
    stats = st.as_dict()
    if segmented:
        in_row = 4 + 4 + 8
        out_row = 4 + 4 + 8 * 4
    elif workload.startswith("cdistinct_"):
        in_row, out_row = 8, 4 + 8 + 8
    else:
        in_row = 8 + (8 if aggs & (isa.ISA_SUM_I64 | isa.ISA_MIN_I64 | isa.ISA_MAX_I64) else 0) + (8 if with_f else 0)
        out_row = row_b
    # algorithmic HBM bytes of a step: every input column read once, every
    # output row written once (runs crossing the host link are counted apart)
    algo_bytes = n * in_row + groups * out_row
    achieved = algo_bytes / (ms_per_step * 1e-3) / 1e9
    traffic = step_traffic(workload)
    roofline = {"bound": "hbm", "scope": "whole step", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
                "algo_bytes_per_step": int(algo_bytes),
                "traffic": int(traffic) if traffic else None,
                "traffic_over_algo": round(traffic / algo_bytes, 2) if traffic else None}
    res = {"ms_per_step": round(ms_per_step, 3), "rows_per_s": round(n / (ms_per_step * 1e-3), 1),
           "groups": groups, "roofline": roofline, "steps": steps, "warmup": warmup,
           "config": {"workload": workload, "rows": n, "distinct_domain": d, "zipf_s": s,
                      "budget_bytes": budget, "aggs": aggs_name, "groups": groups,
                      "run_generation": "replacement" if workload.endswith("_rs") else "read-sort-write"},
           "dtype": "u64+i64+f64" if with_f else ("i32+i32+i64" if segmented else "u64+i64")}
    if stats["spilled_rows"] or spilling:
        res["stats"] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()}
        res["phases_timed_ms"] = timed_phases
    if detail:
        # per-kernel HIP-event timing in separate calls, so that the event
        # records do not enter the timed calls above
        prof = {}
        if args.profile_steps:
            ctx.profile(True)
            for i in range(args.profile_steps):
                step()
            torch.cuda.synchronize()
            prof = ctx.profile_read()
            ctx.profile(False)
            print("bench: %d profiled call(s) done" % args.profile_steps, file=sys.stderr, flush=True)
        kernels = {}
        for name, r in prof.items():
            kernels[name] = {"launches": r["launches"] / args.profile_steps,
                             "avg_us": round(1e3 * r["total_ms"] / max(1, r["launches"]), 2),
                             "ms_per_step": round(r["total_ms"] / args.profile_steps, 3)}
        res["kernels_event_timed"] = kernels
        dom = rocprof_dominant(workload)
        if dom:
            name, avg_us, per_step = dom
            label = next((lb for lb, ks in KERNELS_OF_LABEL.items() if name in ks), name)
            ev = kernels.get(label)
            dk = {"name": name, "source": "committed rocprofv3 summary (same kernel source)",
                  "rocprof_avg_us": avg_us, "launches_per_step": round(per_step, 1),
                  "event_avg_us": ev["avg_us"] if ev else None,
                  "share_of_step": round(avg_us * per_step / (ms_per_step * 1e3), 3)}
            # its HBM rate from the committed counters (FETCH_SIZE + WRITE_SIZE
            # per launch over rocprof's average duration of the same source)
            t = _profiles("hbm_traffic.json")
            c = (t or {}).get("workloads", {}).get(workload, {}).get(name)
            if c:
                gbs = (c["fetch_bytes_per_launch"] + c["write_bytes_per_launch"]) / (avg_us * 1e-6) / 1e9
                dk["counter_GBps"] = round(gbs, 1)
                dk["counter_frac_of_hbm_peak"] = round(gbs / HBM_PEAK_GBS, 4)
            # a kernel that reads host memory is bound by the link: its host
            # bytes per launch (from the library's own launch records) over
            # rocprof's average duration
            if label in prof and label == "merge_h2d" and prof[label]["launches"]:
                hb = prof[label]["bytes"] / prof[label]["launches"]
                dk["host_bytes_per_launch"] = int(hb)
                dk["link_GBps"] = round(hb / (avg_us * 1e-6) / 1e9, 1)
                dk["link_frac"] = round(hb / (avg_us * 1e-6) / 1e9 / LINK_PEAK_GBS, 3)
            roofline["dominant_kernel"] = dk
        if stats["spilled_rows"]:
            hl_ms = sum(prof[k]["total_ms"] for k in ("spill_d2h", "merge_h2d") if k in prof) / max(1, args.profile_steps)
            res["host_link"] = link_summary(stats["spilled_bytes"], hl_ms, ms_per_step)
            # the combined floor: HBM bytes at peak or both link volumes at the link's peak
            floor = max(algo_bytes / (HBM_PEAK_GBS * 1e9), 2 * stats["spilled_bytes"] / (LINK_PEAK_GBS * 1e9)) * 1e3
            roofline["combined_floor_ms"] = round(floor, 3)
            roofline["frac_of_combined_floor"] = round(floor / ms_per_step, 4)
        if args.cpu_sample and not segmented and not workload.startswith("cdistinct_"):
            one, par = cpu_oracle(a0, a1, a2, n, args.cpu_sample, not args.no_parallel_oracle)
            res["cpu_baseline"] = one
            res["cpu_baseline_parallel"] = par
            res["host"] = host_info()
    del a0, a1, a2, ws, spill, outs
    ctx.close()
    torch.cuda.empty_cache()
    return res


# the other configurations reported beside the headline, with fewer calls
SIDE_WORKLOADS = ["plain_1M_10k", "spill_100M_zipf0", "spill_100M_zipf1.2", "nospill_100M_zipf0.8",
                  "segmented_200M"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="spill_100M_zipf0.8", choices=sorted(WORKLOADS) + list(FORMS))
    ap.add_argument("--only", action="store_true",
                    help="the named workload alone (default for the headline: every configuration)")
    ap.add_argument("--side-steps", type=int, default=3, help="timed calls of each side configuration")
    ap.add_argument("--instances", type=int, default=10000, help="batch_*: number of instances")
    ap.add_argument("--requests", type=int, default=2000, help="serve_c4: number of requests")
    ap.add_argument("--rho", type=float, default=0.8, help="serve_c4: offered load vs the plain rate")
    ap.add_argument("--slots", type=int, default=3, help="serve_c4: concurrent server batches")
    ap.add_argument("--tuning-file", default=None,
                    help="batch_*: JSON table of autotuned launch configurations (read, and written when tuning)")
    ap.add_argument("--cpu-sample", type=int, default=20_000_000,
                    help="rows of the input the single-threaded CPU oracle is timed on (0 = skip the oracle)")
    ap.add_argument("--no-parallel-oracle", action="store_true", help="skip the multi-threaded oracle timing")
    ap.add_argument("--profile-steps", type=int, default=2,
                    help="extra untimed calls with per-kernel HIP-event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU (--gpus %d requested); "
              "multi-GPU sharding is a design note, not built" % args.gpus, file=sys.stderr)
        sys.exit(2)
    t_start = time.perf_counter()

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

    if args.workload in FORMS:
        if args.workload == "serve_c4":
            r = bench_serve(args)
        else:
            r = bench_batch(args, 1e3, 1e7 if args.workload == "batch_c3" else 1e5)
        r["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
        print(json.dumps(r))
        return

    head = run_workload(args, args.workload, args.steps, args.warmup, detail=True)
    res = {
        "metric": "input rows/s aggregated (% HBM roofline)",
        "value": head["rows_per_s"],
        "unit": "rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head.get("cpu_baseline"),
    }
    for k in ("cpu_baseline_parallel", "host", "host_link", "stats", "phases_timed_ms", "kernels_event_timed"):
        if k in head:
            res[k] = head[k]
    if not args.only and args.workload == "spill_100M_zipf0.8":
        side = {}
        for w in SIDE_WORKLOADS:
            r = run_workload(args, w, args.side_steps, 1, detail=False)
            side[w] = {k: r[k] for k in ("ms_per_step", "rows_per_s", "groups", "roofline") if k in r}
            if "stats" in r:
                side[w]["runs"] = r["stats"]["runs"]
                side[w]["spilled_rows"] = r["stats"]["spilled_rows"]
            print("bench: %s %.3f ms" % (w, r["ms_per_step"]), file=sys.stderr, flush=True)
        args.workload = "batch_c3"
        b = bench_batch(args, 1e3, 1e7)
        side["batch_c3"] = {k: b[k] for k in ("batched_tuned_rows_per_s", "batched_default_config_rows_per_s",
                                              "plain_per_instance_rows_per_s", "speedup_vs_plain", "ms",
                                              "tuning", "config")}
        args.workload = "serve_c4"
        sv = bench_serve(args)
        side["serve_c4"] = {k: sv[k] for k in ("server", "fifo_plain", "plain_rate_rows_per_s", "config")}
        res["configs"] = side
    res["bench_wall_s"] = round(time.perf_counter() - t_start, 1)
    print(json.dumps(res))


if __name__ == "__main__":
    main()

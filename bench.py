#!/usr/bin/env python3
"""Benchmark of the join hot path on one MI355X.

Workload (default): the large PK-FK join of the paper's wide-join experiments
(Section 5.1): |R| = 2^27 (keys a random permutation of 0..2^27-1), |S| = 2^28
foreign keys uniform over R's keys (match ratio 100%), 4 int32 payload columns
per side, GFTR materialization. One step = one gj_join call: histogram, scan and
stable scatter of both relations (two passes), work units, LDS hash build and
probe (count pass), output sizing, and the write pass that materializes
(key, 4 R payloads, 4 S payloads) for all 2^28 output rows. Output allocation
is inside the step (torch's caching allocator, warm after the first step).

Prints one JSON line. `value` is materialized join tuples/s (|T| / time). The
roofline object is for the kernel with the largest total time in the timed
region: its algorithmic bytes (compulsory reads + writes, computed by the
library per launch) over its HIP-event-measured time on the library's stream.
The CPU baseline is the plain oracle (single thread) on a smaller sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_info() -> dict:
    """CPU model, logical CPUs usable by this process, and host RAM."""
    model = "unknown"
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
    return {"cpu_model": model, "cpus_available": len(os.sched_getaffinity(0)), "host_ram_gib": ram}


def cpu_baseline(payloads: int = 4, log2_1t: int = 22, log2_mt: int = 24, threads: int = 0) -> dict:
    """The plain CPU oracle on bounded samples of the benchmark's workload:
    Oracle-1T (one thread) and Oracle-MT (`threads` threads, default the usable
    CPUs up to 16, each joining one key-hash shard of R and S with the same
    oracle; equi-join decomposes exactly over key shards). Compute only."""
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import datagen
    import oracle
    oracle.build(force=False)
    info = host_info()
    k = threads or max(1, min(16, info["cpus_available"]))

    def sample(lg):
        return datagen.pk_fk_join(1 << lg, 1 << (lg + 1), payloads, payloads, seed=datagen.seed_for(1, 500 + lg))

    d = sample(log2_1t)
    t0 = time.perf_counter()
    cols = oracle.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"])
    dt1 = time.perf_counter() - t0
    one = {"value": len(cols[0]) / dt1, "seconds": dt1, "cores": 1,
           "sample": f"|R|=2^{log2_1t}, |S|=2^{log2_1t + 1}"}
    del cols, d

    d = sample(log2_mt)
    t0 = time.perf_counter()
    with np.errstate(over="ignore"):
        hr = (d["r_key"].astype(np.uint32) * np.uint32(0x9E3779B1)) >> np.uint32(24)
        hs = (d["s_key"].astype(np.uint32) * np.uint32(0x9E3779B1)) >> np.uint32(24)
    shard_r, shard_s = hr % k, hs % k

    def part(i):
        mr, ms = shard_r == i, shard_s == i
        out = oracle.join(d["r_key"][mr], [p[mr] for p in d["r_pay"]], d["s_key"][ms], [p[ms] for p in d["s_pay"]])
        return len(out[0])

    with ThreadPoolExecutor(max_workers=k) as ex:
        t_rows = sum(ex.map(part, range(k)))
    dtm = time.perf_counter() - t0
    assert t_rows == 1 << (log2_mt + 1)
    return {"value": t_rows / dtm, "unit": "tuples/s", "cores": k, "kind": "oracle",
            "sample": f"PK-FK join |R|=2^{log2_mt}, |S|=2^{log2_mt + 1}, {payloads}+{payloads} int32 payloads, "
                      f"uniform FK, mr=100%: Oracle-MT, {k} threads over {k} key-hash shards, {dtm:.1f} s "
                      f"(qsort + binary search per shard)",
            "oracle_1t": dict(one, unit="tuples/s",
                              note="the same oracle single-threaded (qsort + binary search)"),
            "host": info}


def copy_ceiling(nbytes: int = 1 << 31, reps: int = 5, use_torch: bool = False) -> float:
    """Bandwidth of a plain device copy (read n + write n bytes), in GB/s, with
    the library's streaming kernel (or torch's copy): the practical ceiling for
    streaming kernels, and the kernel the HBM counters are calibrated against."""
    import torch
    import paper_2312_00720_amd as gj
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    run = (lambda: y.copy_(x)) if use_torch else (lambda: gj.stream_copy(x, y))
    run()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    if not use_torch:
        assert torch.equal(x, y)
    del x, y
    return 2.0 * nbytes / (ms / 1e3) / 1e9


def bench_micro(args, copy_gbs) -> int:
    """The machine constants of the cost model (Section 4.1.1, Table 1): the
    library's stream copy, and 2^27 4-byte gathers with a clustered map (a random
    permutation inside every 2048-row block, as after radix partitioning) and an
    unclustered one (a random permutation of all rows). With s = unclustered /
    clustered time, B_G / B_R = (12 s - 8) / 4. Also the paper's end-to-end
    comparison: partitioning (key, value) and a clustered gather against the
    unclustered gather alone."""
    import torch
    import paper_2312_00720_amd as gj
    n = 1 << args.gather_log2
    g = torch.Generator(device="cuda")
    g.manual_seed(231200720)
    vals = torch.randint(-2**31, 2**31 - 1, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
    unclustered = torch.randperm(n, generator=g, device="cuda").to(torch.int32)
    blk = 2048
    local = torch.argsort(torch.rand(n, generator=g, device="cuda").view(-1, blk), dim=1)
    clustered = (local + torch.arange(0, n, blk, device="cuda").view(-1, 1)).flatten().to(torch.int32)
    del local
    out = torch.empty(n, dtype=torch.int32, device="cuda")

    def ms_of(fn, reps=args.steps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    t_u = ms_of(lambda: gj.gather_i32(unclustered, vals, out))
    assert torch.equal(out, vals[unclustered.long()])
    t_c = ms_of(lambda: gj.gather_i32(clustered, vals, out))
    assert torch.equal(out, vals[clustered.long()])
    s_ratio = t_u / t_c
    keys = unclustered  # the tuple ids the GFUR gather would use, as a key column
    t_p = ms_of(lambda: gj.partition(keys, [vals], bits=14, passes=2))
    copy_torch = copy_ceiling(use_torch=True)
    res = {
        "metric": "gather ms (2^%d x 4 B)" % args.gather_log2, "value": t_u, "unit": "ms",
        "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": t_u, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"clustered vs unclustered gather of 2^{args.gather_log2} int32 values "
                               f"(clustered: permutation within {blk}-row blocks)"},
        "stream_copy_gbs": copy_gbs, "torch_copy_gbs": copy_torch,
        "gather_unclustered_ms": t_u, "gather_clustered_ms": t_c, "time_ratio": s_ratio,
        "bg_over_br": (12.0 * s_ratio - 8.0) / 4.0,
        "gather_clustered_gbs": 12.0 * n / (t_c / 1e3) / 1e9,
        "gather_unclustered_gbs": 12.0 * n / (t_u / 1e3) / 1e9,
        "partition_14bit_ms": t_p,
        "partition_plus_clustered_speedup": t_u / (t_p + t_c),
        "roofline": {"bound": "hbm", "kernel": "k_gather (clustered)", "achieved": 12.0 * n / (t_c / 1e3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": 12.0 * n / (t_c / 1e3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": None, "alg_bytes_per_launch": 12.0 * n, "avg_launch_ms": t_c},
    }
    print(json.dumps(res), flush=True)
    return 0


GB_AGGS = [(0, "count"), (0, "sum"), (0, "min"), (0, "max"), (1, "sum"), (1, "min"), (1, "max")]
# The paper's own group-by benchmark aggregates MAX of both value columns (§5.2).
GB_AGGS_MAX = [(0, "max"), (1, "max")]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes (profiles/traffic.json), or None when there is
    no such measurement or any source it depends on (the kernels, the launch
    rules) has changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    e = json.load(open(path)).get(f"{kernel}@{workload}")
    if not e:
        return None
    # every source that shapes the measured launches (kernel and launch rules)
    for rel, sha in e["sources"].items():
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src) or hashlib.sha256(open(src, "rb").read()).hexdigest() != sha:
            return None
    return e["hbm_bytes_per_launch"]


def timed(step, steps, warmup):
    """Warm up, time `steps` calls (no per-launch events: wall clock between two
    device synchronizations), then run `steps` more calls with per-launch HIP
    events for the kernel breakdown. Returns (ms per step of the plain run,
    per-kernel stats of the profiled run, ms per step of the profiled run, the
    last output)."""
    import torch
    import paper_2312_00720_amd as gj
    out = None
    for _ in range(warmup):
        out = step()
        del out
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    del out
    gj.profile_start()
    t2 = time.perf_counter()
    for _ in range(steps):
        out = step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stats = gj.profile_stop()
    return (t1 - t0) / steps * 1e3, stats, (t3 - t2) / steps * 1e3, out


def kernel_table(stats, steps):
    kern = {k: dict(v, ms_per_step=v["total_ms"] / steps,
                    gbs=(v["alg_bytes"] / (v["total_ms"] / 1e3) / 1e9) if v["total_ms"] > 0 else 0.0)
            for k, v in stats.items()}
    return dict(sorted(kern.items(), key=lambda x: -x[1]["total_ms"]))


def roofline(dom, dk, traffic=None,
             source="HIP events around every launch of the profiled run, on the library's stream"):
    """Roofline object of the dominant kernel: algorithmic bytes per launch over
    its average launch time (both from per-launch HIP events)."""
    return {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
            "alg_bytes_per_launch": dk["alg_bytes"] / max(1, dk["launches"]),
            "avg_launch_ms": dk["total_ms"] / max(1, dk["launches"]),
            "source": source}


def bench_groupby(args, copy_gbs) -> int:
    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    n, g = 1 << args.n_log2, 1 << args.g_log2
    log(f"generating group-by N=2^{args.n_log2} g=2^{args.g_log2} alpha={args.alpha}")
    d = dd.groupby_input(n, g, 2, seed=datagen.seed_for(2, args.g_log2), alpha=args.alpha)
    keys_desc = "int32 key"
    if args.gb_key_bytes == 8:
        # 8-byte keys: the values 0..g-1 through an odd multiplier, so all 8 bytes vary
        d["key"] = d["key"].to(torch.int64) * -7046029254386353131  # 0x9E3779B97F4A7C15 as int64
        keys_desc = "int64 key (g values spread over all 8 bytes)"
    elif args.sparse_keys:
        # an odd multiplier is a bijection modulo 2^32: g distinct keys whose 4 bytes all vary
        d["key"] = ((d["key"].to(torch.int64) * 0x9E3779B1) & 0xFFFFFFFF).to(torch.int32)
        keys_desc = "int32 key (g values spread over all 4 bytes)"
    torch.cuda.synchronize()
    mat = args.mat if args.algo not in ("hash", "auto") else "auto"

    aggs = GB_AGGS if args.gb_aggs == "all" else GB_AGGS_MAX

    def step():
        return gj.groupby(d["key"], d["vals"], aggs, algo=args.algo, mat=mat, radix_bits=args.radix_bits)

    ms, stats, ms_prof, out = timed(step, args.steps, args.warmup)
    groups = out[0].numel()
    kern = kernel_table(stats, args.steps)
    dom = next(iter(kern))
    dk = kern[dom]
    res = {
        "metric": "group-by rows/s", "value": n / (ms / 1e3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"group-by N=2^{args.n_log2}, {keys_desc} over 2^{args.g_log2} values "
                               f"({'uniform' if args.alpha == 0 else f'zipf {args.alpha}'}), 2 int32 values, "
                               f"{'COUNT+SUM+MIN+MAX' if args.gb_aggs == 'all' else 'MAX'}, {args.algo}"
                               + ("" if args.algo == "hash" else f" {mat.upper()}"),
                   "groups": groups},
        "copy_ceiling_gbs": copy_gbs,
        "roofline": roofline(dom, dk,
                             measured_traffic(dom, f"groupby_{args.algo}_n{args.n_log2}_g{args.g_log2}")
                             if args.alpha == 0 and mat in ("gftr", "auto") and args.radix_bits == 0
                             and keys_desc == "int32 key" and args.gb_aggs == "all" else None),
        "hbm_gbs_whole_step": sum(v["alg_bytes"] for v in stats.values()) / args.steps / (ms / 1e3) / 1e9,
        "profiled_ms_per_step": ms_prof,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["ms_per_step"],
                        "alg_gbs": v["gbs"]} for k, v in kern.items()},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_pipeline(args, copy_gbs) -> int:
    """Join then group-by: R = 2^16 rows (keys a permutation, one int32 payload),
    S = 2^26 foreign keys with one int32 payload; the join output is grouped on
    its R payload (about 2^16 groups) with COUNT, SUM, MIN and MAX of the S payload."""
    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    n_r, n_s = 1 << 16, 1 << args.pipe_s_log2
    d = dd.pk_fk_join(n_r, n_s, 1, 1, seed=datagen.seed_for(2, 900))
    torch.cuda.synchronize()
    aggs = [(0, "count"), (0, "sum"), (0, "min"), (0, "max")]

    def step():
        k, rp, sp = gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat=args.mat)
        return gj.groupby(rp[0], [sp[0]], aggs, algo="auto")

    ms, stats, ms_prof, out = timed(step, args.steps, args.warmup)
    kern = kernel_table(stats, args.steps)
    dom = next(iter(kern))
    dk = kern[dom]
    res = {
        "metric": "join + group-by input rows/s", "value": n_s / (ms / 1e3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"PK-FK join |R|=2^16 |S|=2^{args.pipe_s_log2} (1+1 int32 payloads, {args.mat.upper()}) "
                               "then group-by on the R payload, COUNT/SUM/MIN/MAX of the S payload, algorithm auto",
                   "groups": int(out[0].numel())},
        "copy_ceiling_gbs": copy_gbs,
        "roofline": roofline(dom, dk),
        "profiled_ms_per_step": ms_prof,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["ms_per_step"],
                        "alg_gbs": v["gbs"]} for k, v in kern.items()},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_batch(args, copy_gbs) -> int:
    """Batched PK-FK joins: one plan captured into a HIP graph and launched once per
    step, against one gj_join call per instance (same inputs, same stream)."""
    import numpy as np
    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    n = args.instances
    r_sz, s_sz = datagen.batch_sizes(n, datagen.seed_for(3, n))
    log(f"generating {n} instances: sum|R|={int(r_sz.sum())} sum|S|={int(s_sz.sum())}")
    d = dd.join_batch(r_sz, s_sz, 2, datagen.seed_for(3, n + 1))
    torch.cuda.synchronize()
    cols = (d["r_key"], d["r_pay"], d["r_off"], d["s_key"], d["s_pay"], d["s_off"])
    tuning = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        tuning = gj.join_autotune(*cols, mat=args.mat, reps=3)
        log(f"autotuned in {time.perf_counter() - t0:.1f} s: {gj.tuning_dict(tuning)}")
    plan = gj.JoinPlan(*cols, mat=args.mat, tuning=tuning)
    info = plan.info()
    log(f"plan: {info}")
    plan.capture()
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    key, rp, sp, off = plan.result()
    T = key.numel()
    assert T == int(s_sz.sum()) and off[-1] == T, "every S row matches exactly once"
    log(f"graph: {ms:.2f} ms per batch, |T| = {T}")
    # per-kernel times from one eager run of the same plan (the graph hides them)
    gj.profile_start()
    plan.run()
    torch.cuda.synchronize()
    stats = gj.profile_stop()
    kern = kernel_table(stats, 1)
    dom = next(iter(kern))
    dk = kern[dom]
    # one gj_join call per instance on the same columns
    r_off, s_off = d["r_off"], d["s_off"]

    def one(i):
        return gj.join(d["r_key"][r_off[i]:r_off[i + 1]], [x[r_off[i]:r_off[i + 1]] for x in d["r_pay"]],
                       d["s_key"][s_off[i]:s_off[i + 1]], [x[s_off[i]:s_off[i + 1]] for x in d["s_pay"]],
                       mat=args.mat)
    for i in range(min(n, 32)):
        one(i)  # warm-up of the allocator and the library
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_single = 0
    for i in range(n):
        o = one(i)
        t_single += o[0].numel()
        del o
        if (i + 1) % 1024 == 0:
            log(f"per-instance calls: {i + 1}/{n}")
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3
    assert t_single == T
    # launch count of the per-instance calls, from a separate profiled pass
    gj.profile_start()
    for i in range(n):
        del_o = one(i)
        del del_o
    torch.cuda.synchronize()
    single_launches = sum(v["launches"] for v in gj.profile_stop().values())
    plan.close()
    res = {
        "metric": "materialized join tuples/s", "value": T / (ms / 1e3), "unit": "tuples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch of {n} PK-FK joins, |R_i| = round(2^U(8,20)), |S_i| = m_i|R_i|, "
                               f"m_i in 4..16, 2+2 int32 payloads, {args.mat.upper()}, one HIP graph launch",
                   "sum_r": int(r_sz.sum()), "sum_s": int(s_sz.sum()), "output_rows": T,
                   "tuning": gj.tuning_dict(tuning) if tuning is not None else None},
        "plan": info,
        "per_instance": {"ms": ms_single, "tuples_per_s": T / (ms_single / 1e3), "launches": single_launches},
        "speedup_vs_per_instance": ms_single / ms,
        "copy_ceiling_gbs": copy_gbs,
        "roofline": roofline(dom, dk, source="one eager run of the plan with per-launch events"),
        "kernels": {k: {"launches": v["launches"], "ms": v["ms_per_step"], "alg_gbs": v["gbs"]}
                    for k, v in kern.items()},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_gbbatch(args, copy_gbs) -> int:
    """Batched partition group-bys: one plan captured into a HIP graph and launched
    once per step, against one gj_groupby call per instance (same inputs, same
    stream). Instance i has N_i = round(2^U(8,20)) rows, keys uniform over
    max(4, N_i / 16) values, 2 int32 values, COUNT+SUM+MIN+MAX."""
    import numpy as np
    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    n = args.instances
    sizes, _ = datagen.batch_sizes(n, datagen.seed_for(4, n))
    cards = np.maximum(4, sizes >> 4)
    log(f"generating {n} group-by instances: sum N = {int(sizes.sum())}")
    d = dd.groupby_batch(sizes, cards, 2, datagen.seed_for(4, n + 1))
    torch.cuda.synchronize()
    off = d["off"]
    plan = gj.GroupByPlan(d["key"], d["vals"], off, GB_AGGS, mat=args.mat)
    info = plan.info()
    log(f"plan: {info}")
    plan.capture()
    for _ in range(args.warmup):
        plan.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    keys, _, goff = plan.result()
    G = keys.numel()
    log(f"graph: {ms:.2f} ms per batch, {G} groups")
    gj.profile_start()
    plan.run()
    torch.cuda.synchronize()
    kern = kernel_table(gj.profile_stop(), 1)
    dom = next(iter(kern))
    dk = kern[dom]

    def one(i):
        return gj.groupby(d["key"][off[i]:off[i + 1]], [v[off[i]:off[i + 1]] for v in d["vals"]], GB_AGGS,
                          algo="partition", mat=args.mat)
    for i in range(min(n, 32)):
        one(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g_single = 0
    for i in range(n):
        o = one(i)
        g_single += o[0].numel()
        del o
        if (i + 1) % 1024 == 0:
            log(f"per-instance calls: {i + 1}/{n}")
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t0) * 1e3
    gj.profile_start()
    for i in range(n):
        del_o = one(i)
        del del_o
    torch.cuda.synchronize()
    single_launches = sum(v["launches"] for v in gj.profile_stop().values())
    assert g_single == G and goff[-1] == G, "the plan and the per-instance calls find the same groups"
    plan.close()
    rows = int(sizes.sum())
    res = {
        "metric": "group-by rows/s", "value": rows / (ms / 1e3), "unit": "rows/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"batch of {n} partition group-bys, N_i = round(2^U(8,20)), keys uniform over "
                               f"max(4, N_i/16) values, 2 int32 values, COUNT+SUM+MIN+MAX, {args.mat.upper()}, "
                               f"one HIP graph launch", "sum_rows": rows, "groups": G},
        "plan": info,
        "per_instance": {"ms": ms_single, "rows_per_s": rows / (ms_single / 1e3), "launches": single_launches},
        "speedup_vs_per_instance": ms_single / ms,
        "copy_ceiling_gbs": copy_gbs,
        "roofline": roofline(dom, dk, source="one eager run of the plan with per-launch events"),
        "kernels": {k: {"launches": v["launches"], "ms": v["ms_per_step"], "alg_gbs": v["gbs"]}
                    for k, v in kern.items()},
    }
    print(json.dumps(res), flush=True)
    return 0


def bench_sweep(args, copy_gbs) -> int:
    """The join sweeps of Section 5.1, one JSON line per point, every point run
    with partitioned hash join and sort-merge join under GFTR and GFUR:
      m2n:      |R| = |S| = 2^26, keys uniform over |K| in {2^23, 2^24, 2^25}
                unique values, 2 int32 payload columns per side (many-to-many);
      ratio:    |S| = 2^27 PK-FK, |R| = 2^21 .. 2^27, 2 payload columns per side;
      payloads: |R| = |S| = 2^27 PK-FK, 1, 2, 4 or 8 payload columns per side."""
    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj
    algos = [("phj", "gftr"), ("phj", "gfur"), ("smj", "gftr"), ("smj", "gfur")]

    def m2n_inputs(n, k, c, seed):
        g = dd.generator(seed)
        rk = torch.randint(0, k, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        sk = torch.randint(0, k, (n,), generator=g, device="cuda", dtype=torch.int64).to(torch.int32)
        return {"r_key": rk, "s_key": sk, "r_pay": dd.payloads(g, n, c), "s_pay": dd.payloads(g, n, c)}

    points = []
    if args.sweep in ("all", "m2n"):
        points += [("m2n", dict(n_r=1 << 26, n_s=1 << 26, c=2, k=1 << kk)) for kk in (23, 24, 25)]
    if args.sweep in ("all", "ratio"):
        points += [("ratio", dict(n_r=1 << lr, n_s=1 << 27, c=2)) for lr in (21, 23, 25, 27)]
    if args.sweep in ("all", "payloads"):
        points += [("payloads", dict(n_r=1 << 27, n_s=1 << 27, c=c)) for c in (1, 2, 4, 8)]
    for name, pt in points:
        if name == "m2n":
            d = m2n_inputs(pt["n_r"], pt["k"], pt["c"], datagen.seed_for(1, 700 + pt["k"].bit_length()))
        else:
            d = dd.pk_fk_join(pt["n_r"], pt["n_s"], pt["c"], pt["c"],
                              seed=datagen.seed_for(1, 800 + pt["n_r"].bit_length() + 40 * pt["c"]))
        torch.cuda.synchronize()
        res = {"sweep": name, **pt, "unit": "ms", "runs": {}}
        for algo, mat in algos:
            def step():
                return gj.join(d["r_key"], d["r_pay"], d["s_key"], d["s_pay"], mat=mat, algo=algo)
            out = step()
            t_rows = out[0].numel()
            del out
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                out = step()
                del out
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / args.steps * 1e3
            res["runs"][f"{algo}-{mat}"] = {"ms": ms, "output_rows": t_rows, "tuples_per_s": t_rows / (ms / 1e3)}
            log(f"sweep {name} {pt} {algo}-{mat}: {ms:.2f} ms, |T| = {t_rows}")
        print(json.dumps(res), flush=True)
        del d
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mat", default="gftr", choices=["gftr", "gfur"])
    ap.add_argument("--join-algo", default="phj", choices=["phj", "smj"], help="join: partitioned hash or sort-merge")
    ap.add_argument("--r-log2", type=int, default=27)
    ap.add_argument("--s-log2", type=int, default=28)
    ap.add_argument("--payloads", type=int, default=4)
    ap.add_argument("--key-bytes", type=int, default=4, choices=[4, 8])
    ap.add_argument("--alpha", type=float, default=0.0)
    ap.add_argument("--match-ratio", type=float, default=1.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--radix-bits", type=int, default=0, help="join / group-by: partition bits (0 = automatic)")
    ap.add_argument("--lds-budget", type=int, default=0, help="join: max R rows per build block (0 = automatic)")
    ap.add_argument("--workload", default="join",
                    choices=["join", "groupby", "batch", "gbbatch", "pipeline", "micro", "sweep"])
    ap.add_argument("--sweep", default="all", choices=["all", "m2n", "ratio", "payloads"],
                    help="sweep workload: which join sweep of Section 5.1")
    ap.add_argument("--gather-log2", type=int, default=27, help="micro: gathered values")
    ap.add_argument("--pipe-s-log2", type=int, default=26, help="pipeline: log2 |S|")
    ap.add_argument("--instances", type=int, default=4096, help="batch: join instances")
    ap.add_argument("--no-autotune", action="store_true", help="batch: built-in plan parameters")
    ap.add_argument("--n-log2", type=int, default=28, help="group-by rows")
    ap.add_argument("--g-log2", type=int, default=16, help="group-by key cardinality")
    ap.add_argument("--sparse-keys", action="store_true", help="group-by: spread the keys over all 4 bytes")
    ap.add_argument("--gb-key-bytes", type=int, default=4, choices=[4, 8], help="group-by key width")
    ap.add_argument("--gb-aggs", default="all", choices=["all", "max"],
                    help="group-by aggregates: COUNT+SUM+MIN+MAX of both columns, or MAX of both (the paper's)")
    ap.add_argument("--algo", default="partition", choices=["partition", "hash", "sort", "sort_de", "auto"])
    ap.add_argument("--copy-only", action="store_true",
                    help="only run the plain copy (counter calibration) and print its GB/s")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the join and group-by "
              "run on a single device and no multi-GPU path is built.", file=sys.stderr)
        return 2

    import torch
    import datagen
    import datagen.device as dd
    import paper_2312_00720_amd as gj

    if args.copy_only:
        print(json.dumps({"copy_gbs": copy_ceiling(), "bytes_each_way": 1 << 31}), flush=True)
        return 0
    copy_gbs = copy_ceiling()
    log(f"plain copy: {copy_gbs:.0f} GB/s")

    if args.workload == "groupby":
        return bench_groupby(args, copy_gbs)
    if args.workload == "gbbatch":
        return bench_gbbatch(args, copy_gbs)
    if args.workload == "batch":
        return bench_batch(args, copy_gbs)
    if args.workload == "pipeline":
        return bench_pipeline(args, copy_gbs)
    if args.workload == "micro":
        return bench_micro(args, copy_gbs)
    if args.workload == "sweep":
        return bench_sweep(args, copy_gbs)

    n_r, n_s, c = 1 << args.r_log2, 1 << args.s_log2, args.payloads
    log(f"generating |R|=2^{args.r_log2} |S|=2^{args.s_log2} payloads={c} key_bytes={args.key_bytes}")
    d = dd.pk_fk_join(n_r, n_s, c, c, seed=datagen.seed_for(1), alpha=args.alpha,
                      match_ratio=args.match_ratio, key_bytes=args.key_bytes)
    torch.cuda.synchronize()
    rk, rp, sk, sp = d["r_key"], d["r_pay"], d["s_key"], d["s_pay"]

    def step():
        return gj.join(rk, rp, sk, sp, mat=args.mat, radix_bits=args.radix_bits, lds_budget=args.lds_budget,
                       algo=args.join_algo)

    n_out = None
    for i in range(args.warmup):
        out = step()
        n_out = out[0].numel()
        del out
        log(f"warmup {i + 1}/{args.warmup} done (|T| = {n_out})")
    torch.cuda.synchronize()

    # the timed region: no per-launch events, wall clock between synchronizations
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step()
        n_out = out[0].numel()
        del out
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed {args.steps} steps")
    # the same number of steps again with per-launch HIP events on the library's
    # stream: the kernel breakdown and the roofline come from this run
    gj.profile_start()
    t2 = time.perf_counter()
    for i in range(args.steps):
        out = step()
        del out
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stats = gj.profile_stop()
    log(f"profiled {args.steps} steps")

    ms = (t1 - t0) / args.steps * 1e3
    value = n_out / (ms / 1e3)
    default_join = (args.r_log2, args.s_log2, c, args.key_bytes, args.alpha, args.match_ratio, args.mat,
                    args.radix_bits, args.lds_budget, args.join_algo) == (27, 28, 4, 4, 0.0, 1.0, "gftr", 0, 0, "phj")
    kern = {k: dict(v, ms_per_step=v["total_ms"] / args.steps,
                    gbs=(v["alg_bytes"] / (v["total_ms"] / 1e3) / 1e9) if v["total_ms"] > 0 else 0.0)
            for k, v in stats.items()}
    dom = max(kern, key=lambda k: kern[k]["total_ms"])
    dk = kern[dom]
    alg_total = sum(v["alg_bytes"] for v in stats.values()) / args.steps
    # Phases as the paper counts them (Section 5.1): under GFTR, moving payload
    # columns through the partitioning passes is materialization work. One
    # scatter moves the key and the payloads together, so its time is split by
    # byte share: key (and GFUR row id) bytes to transformation, payload bytes
    # to materialization.
    scatter_ms = sum(kern[k]["ms_per_step"] for k in kern if k.startswith("k_scatter"))
    pay_share = 0.0 if args.mat == "gfur" else (4.0 * c) / (args.key_bytes + 4.0 * c)
    phases = {
        "transform_ms": sum(kern[k]["ms_per_step"] for k in kern
                            if k.startswith(("k_hist", "k_scan", "k_chunk", "k_poff", "k_fill", "k_set")))
        + scatter_ms * (1.0 - pay_share),
        "match_ms": sum(kern[k]["ms_per_step"] for k in kern if k in ("k_unit_count", "k_join_count")),
        "materialize_ms": sum(kern[k]["ms_per_step"] for k in kern if k.startswith("k_join_write"))
        + scatter_ms * pay_share,
        "source": "the profiled run; GFTR payload bytes of the partitioning scatter count as materialization",
    }
    res = {
        "metric": "materialized join tuples/s",
        "value": value,
        "unit": "tuples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32" if args.key_bytes == 4 else "int64",
        "data": "synthetic",
        "config": {"workload": f"PK-FK join |R|=2^{args.r_log2} |S|=2^{args.s_log2}, "
                               f"{c}+{c} int32 payloads, {'int32' if args.key_bytes == 4 else 'int64'} keys, "
                               f"FK {'uniform' if args.alpha == 0 else f'zipf {args.alpha}'}, "
                               f"mr={args.match_ratio:g}, {args.mat.upper()}"
                               + (", sort-merge join" if args.join_algo == "smj" else ""),
                   "n_r": n_r, "n_s": n_s, "payloads_per_side": c, "mat": args.mat,
                   "output_rows": n_out},
        "paper_throughput_rows_per_s": (n_r + n_s) / (ms / 1e3),
        "profiled_ms_per_step": (t3 - t2) / args.steps * 1e3,
        "hbm_gbs_whole_step": alg_total / (ms / 1e3) / 1e9,
        "copy_ceiling_gbs": copy_gbs,
        "roofline": roofline(dom, dk, measured_traffic(dom, "join_default") if default_join else None),
        "phases_ms": phases,
        "kernels": {k: {"launches_per_step": v["launches"] / args.steps, "ms_per_step": v["ms_per_step"],
                        "alg_gbs": v["gbs"]} for k, v in sorted(kern.items(), key=lambda x: -x[1]["total_ms"])},
    }
    if not args.no_cpu_baseline:
        del d, rk, rp, sk, sp
        log("timing the CPU oracle on a bounded sample")
        res["cpu_baseline"] = cpu_baseline(payloads=c)
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())

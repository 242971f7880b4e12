#!/usr/bin/env python3
"""Benchmark of the DF-P update path on one MI355X.

Workload (the large static-graph configuration of the paper's random-batch
experiment, Section 5.2.2, on a synthetic stand-in for its SuiteSparse graphs):
R-MAT scale 24 (a,b,c = 0.57,0.19,0.19), edge factor 16, duplicates removed,
a self-loop on every vertex.  One step = apply one batch of frac*|E| edges
(80% uniform insertions of absent pairs, 20% uniform deletions of existing
edges; batches are chained, each valid against the graph it is applied to)
and update the ranks with DF-P from the previous step's ranks.  Inputs (the
graph and every batch) are resident in device memory before timing starts.

Reported: graph edges per second of whole update steps (|E| / step time), p50
and p99 step latency, the GPU Static (cold) solve time on the same graph, a
roofline figure for the dominant kernel from HIP-event kernel durations inside
the timed region, and the CPU oracle timed on the same first step (same R0,
same batch), which doubles as a full-size parity check.

    python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--scale 24] [--frac 1e-4]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "DF-P update time & edges/s vs GPU Static at L∞ err ≤1e-9; p50/p99 latency"
HBM_PEAK_GBS = 8000.0
# HBM traffic of the pull kernel measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE runs, scaled by a plain-copy calibration), valid for the rank
# engine source it was taken on; see profiles/.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pull_rmat24_dfp_traffic.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def chained_batches(n, src, dst, frac, count, seed):
    """`count` 80/20 batches, each valid against the graph left by the previous ones
    (frac: one fraction of |E| for all, or one per batch).

    Deletions are drawn uniformly among the original edges not yet deleted;
    insertions are uniform pairs u != v absent from the original graph and not
    inserted before."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m_total = src.shape[0] + n
    fracs = list(frac) if hasattr(frac, "__len__") else [frac] * count
    keys0 = src.astype(np.int64) * n + dst.astype(np.int64)
    deleted = np.zeros(src.shape[0], dtype=bool)
    inserted = np.empty(0, dtype=np.int64)
    out = []
    for step in range(count):
        b = max(1, int(round(fracs[step] * m_total)))
        b_ins = int(round(0.8 * b))
        b_del = min(b - b_ins, src.shape[0])
        sel = np.empty(0, dtype=np.int64)
        while sel.shape[0] < b_del:
            c = rng.integers(0, src.shape[0], size=2 * (b_del - sel.shape[0]) + 8)
            c = c[~deleted[c]]
            c = np.concatenate([sel, c])
            _, first = np.unique(c, return_index=True)
            sel = c[np.sort(first)][:b_del]
        deleted[sel] = True
        ins = np.empty(0, dtype=np.int64)
        while ins.shape[0] < b_ins:
            need = b_ins - ins.shape[0]
            u = rng.integers(0, n, size=need + need // 8 + 8, dtype=np.int64)
            v = rng.integers(0, n, size=u.shape[0], dtype=np.int64)
            k = (u * n + v)[u != v]
            pos = np.minimum(np.searchsorted(keys0, k), keys0.shape[0] - 1)
            k = k[keys0[pos] != k]
            if inserted.shape[0]:
                k = k[~np.isin(k, inserted)]
            k = np.concatenate([ins, k])
            _, first = np.unique(k, return_index=True)
            ins = k[np.sort(first)][:b_ins]
        inserted = np.union1d(inserted, ins)
        out.append((src[sel].copy(), dst[sel].copy(), (ins // n).astype(np.int32), (ins % n).astype(np.int32)))
        if b >= 1_000_000:  # large batches take a while on the host: show progress
            log(f"  batch {step + 1}/{count} drawn ({b} edges)")
    return out


def rank_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("rank.hip", "dfpr_impl.hpp"):
        with open(os.path.join(ROOT, "paper_2401_15870_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_kv(path):
    """`key: value` lines of a profile summary."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(("#", " ", "|", "`")):
                k, v = line.split(":", 1)
                out[k.strip()] = v.strip()
    return out


def measured_traffic(workload_key):
    """Counter-measured HBM bytes per pull launch, or None when the kernel source
    changed since the counters were taken (or none were taken for this workload)."""
    try:
        t = read_kv(TRAFFIC_FILE)
    except OSError:
        return None
    if t.get("source_sha") != rank_source_sha() or t.get("workload") != workload_key:
        return None
    try:
        return float(t["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def device_copy_gbs(torch, dev, nbytes=1 << 30, reps=5):
    """Bytes read + written per second by a device-to-device copy of 1 GiB."""
    a = torch.empty(nbytes // 8, dtype=torch.float64, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


# ---------------------------------------------------------------- profile summaries
def _csv_rows(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name):
    name = name.replace("void ", "")
    return name.split("(")[0]


def summarize_trace(d):
    """Markdown table of a `rocprofv3 --kernel-trace --stats` run (directory d)."""
    import glob
    f = glob.glob(os.path.join(d, "*kernel_stats.csv"))[0]
    rows = _csv_rows(f)
    lines = ["| kernel | calls | total ms | avg us | % |", "|---|---|---|---|---|"]
    for r in rows[:20]:
        lines.append(f"| {_short(r['Name'])} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.1f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    return "\n".join(lines)


def summarize_counters(fetch_dir, write_dir, kernel_prefix):
    """Per-launch HBM bytes of the kernels whose name starts with kernel_prefix,
    from FETCH_SIZE and WRITE_SIZE runs (KiB per dispatch), each scaled by what the
    counter reads for the 1 GiB device copies that end a --calib run."""
    import glob
    out = {}
    for key, d in (("fetch", fetch_dir), ("write", write_dir)):
        rows = _csv_rows(glob.glob(os.path.join(d, "*counter_collection.csv"))[0])
        copies = [r for r in rows if "copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"].lower()]
        copies = copies[-3:]
        kib_copy = sum(float(r["Counter_Value"]) for r in copies) / len(copies)
        factor = (1 << 30) / 1024 / kib_copy
        mine = [float(r["Counter_Value"]) for r in rows if _short(r["Kernel_Name"]).startswith(kernel_prefix)]
        out[key] = {"factor": factor, "launches": len(mine),
                    "kib_per_launch": sum(mine) / max(len(mine), 1)}
    fb = out["fetch"]["kib_per_launch"] * 1024 * out["fetch"]["factor"]
    wb = out["write"]["kib_per_launch"] * 1024 * out["write"]["factor"]
    return out, fb + wb


def pct(a, q):
    return float(np.percentile(np.asarray(a, dtype=np.float64), q))


def batched_members(count, seed, n_lo=1e3, n_hi=1e6):
    """Member graphs of the batched configuration: vertex counts log-uniform in
    [n_lo, n_hi] (default [1e3, 1e6]), edge factor uniform in [8, 32], R-MAT
    draws at scale ceil(log2 n) with endpoints >= n redrawn, duplicates and
    self draws dropped."""
    import workloads as W
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(count):
        n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
        ef = float(rng.uniform(8, 32))
        scale = int(np.ceil(np.log2(n)))
        fr = float(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2))))
        _, s, d = W.rmat_graph(scale, ef, seed=seed * 7919 + k, n_limit=n)
        out.append((n, s, d, fr))
        if (k + 1) % 64 == 0:
            log(f"  generated {k + 1}/{count} member graphs")
    return out


def bench_batched(args):
    """Batched form: every member's apply + DF-P update in one batch handle,
    against the same updates as sequential calls on per-graph handles."""
    import torch
    import paper_2401_15870_amd as dfpr

    dev = torch.device("cuda:0")
    t0 = time.time()
    n_lo, n_hi = (float(x) for x in args.member_n.split(","))
    mem = batched_members(args.graphs, args.seed, n_lo, n_hi)
    total_steps = args.warmup + args.steps
    chains = []
    for k, (n, s, d, fr) in enumerate(mem):
        chains.append(chained_batches(n, s, d, fr, total_steps, seed=args.seed * 104729 + k))
        if (k + 1) % 128 == 0:
            log(f"  batches for {k + 1}/{len(mem)} graphs")
    m_draw = sum(len(s) for _, s, _, _ in mem)
    log(f"batched: {len(mem)} graphs, {sum(n for n, _, _, _ in mem)} vertices, {m_draw} edges "
        f"(no self-loops), gen {time.time() - t0:.1f}s")

    t0 = time.time()
    dmem = [(n, torch.from_numpy(s).to(dev), torch.from_numpy(d).to(dev)) for n, s, d, _ in mem]
    bg = dfpr.BatchGraph.from_coo(dmem)
    if args.batch_loop:
        bg.set_fused_limit(0)  # launch per iteration instead of the single launch
    plain = [dfpr.Graph.from_coo(n, s, d) for n, s, d in dmem]
    del dmem
    torch.cuda.synchronize()
    m_total = bg.m
    log(f"create: arena m={m_total}, {len(plain)} plain handles, {time.time() - t0:.1f}s")
    if not args.no_autotune:
        bounds, ms = bg.autotune()
        for g in plain:
            g.set_tuning(bounds)
        log(f"autotune (arena): {bounds} pull {ms:.3f} ms")
    dev_chains = [[tuple(torch.from_numpy(a).to(dev) for a in b) for b in ch] for ch in chains]

    # R0: per-member Static (cold) computed once on the arena; plain handles start
    # from their slices of the same bits
    r_arena, tot0, _ = bg.update_ranks_many("static", None)
    r_plain = [bg.member(r_arena, k).clone() for k in range(len(plain))]
    log(f"R0: static over the arena, {tot0['iterations']} iterations (slowest member)")

    bg.set_timing(True)
    phases = {"apply": 0.0, "pull": 0.0, "commit": 0.0, "bin": 0.0, "mark": 0.0, "rank_total": 0.0}
    counts = {"pull_launches": 0, "dense_iterations": 0, "edges_pulled": 0, "pull_bytes": 0.0}

    def step_batched(i):
        info = bg.apply_batch_many([dev_chains[k][i] for k in range(len(plain))])
        r, tot, per = bg.update_ranks_many(args.mode, r_arena, out=r_arena)
        if i >= args.warmup:
            phases["apply"] += info[0]["ms_total"]
            phases["pull"] += tot["ms_pull"]
            phases["commit"] += tot["ms_commit"]
            phases["bin"] += tot["ms_bin"]
            phases["mark"] += tot["ms_mark"]
            phases["rank_total"] += tot["ms_total"]
            for key in counts:
                counts[key] += tot[key]
        return info, tot, per

    def step_plain(i):
        its = 0
        for k, g in enumerate(plain):
            g.apply_batch(*dev_chains[k][i])
            _, st = g.update_ranks(args.mode, r_plain[k], out=r_plain[k])
            its += st["iterations"]
        return its

    tb, tp = [], []
    worst = 0.0
    delta_edges = 0
    iters_b = []
    for i in range(total_steps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        info, tot, per = step_batched(i)
        torch.cuda.synchronize()
        t_b = time.perf_counter() - t
        t = time.perf_counter()
        step_plain(i)
        torch.cuda.synchronize()
        t_p = time.perf_counter() - t
        for k in range(len(plain)):
            diff = (bg.member(r_arena, k) - r_plain[k]).abs().max().item() if plain[k].n else 0.0
            worst = max(worst, diff)
        if i >= args.warmup:
            tb.append(t_b)
            tp.append(t_p)
            iters_b.append(tot["iterations"])
            delta_edges += sum(x["ins_in"] + x["del_in"] for x in info)
        log(f"step {i}: batched {t_b * 1e3:.1f} ms (max member iterations {tot['iterations']}), "
            f"sequential {t_p * 1e3:.1f} ms, max |batched - plain| {worst:.3e}")
    assert worst <= 1e-9, f"batched and plain results differ: {worst}"
    K = len(tb)
    tb_s, tp_s = sum(tb), sum(tp)
    G = len(plain)
    res = {
        "metric": "batched DF-P update throughput vs sequential per-graph calls at equal accuracy",
        "value": G * K / tb_s,
        "unit": "graphs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": tb_s * 1e3 / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{G} R-MAT graphs, n log-uniform in [{n_lo:g}, {n_hi:g}], edge factor U[8, 32], one chained "
                               f"80/20 batch of f*|E| per graph per step, f log-uniform in [1e-4, 1e-2]; apply + "
                               f"{args.mode.upper()} update of every graph per step",
                   "graphs": G, "m_total": int(m_total), "mode": args.mode, "parallelism": "1 GPU",
                   # the library's default single-launch limit for batch arenas is 2^26 edges
                   "batch_update": "launch per iteration" if args.batch_loop or m_total > (1 << 26)
                   else "single launch",
                   "bin_bounds": bg.get_tuning()},
        "graph_edges_per_s": m_total * K / tb_s,
        "batch_edges_per_s": delta_edges / tb_s,
        "sequential_ms_per_step": tp_s * 1e3 / K,
        "sequential_graphs_per_s": G * K / tp_s,
        "speedup_vs_sequential": tp_s / tb_s,
        "max_member_iterations_mean": float(np.mean(iters_b)),
        "max_abs_diff_vs_plain": worst,
        "batched_ms_per_step_by_phase": {k: v / K for k, v in phases.items()},
        "batched_counts_per_step": {k: v / K for k, v in counts.items()},
        "pull_achieved_gbs": (counts["pull_bytes"] / (phases["pull"] * 1e-3) / 1e9) if phases["pull"] else None,
    }
    print(json.dumps(res))


SERVING_MIX = ((26, 1), (25, 1), (24, 2), (23, 3), (22, 4), (21, 6), (20, 10), (19, 20), (18, 49))


def bench_serving(args):
    """Serving form: resident R-MAT graphs, Poisson request arrivals, p50/p99
    latency and updates/s with the server's lanes against one lane (FIFO,
    one request at a time) on the same graphs."""
    import threading
    import torch
    import paper_2401_15870_amd as dfpr
    import workloads as W

    mix = [(max(8, sc - args.serving_scale_offset), cnt) for sc, cnt in SERVING_MIX]
    rates = [float(x) for x in args.rates.split(",")]
    per_run = args.requests
    runs = 2 * len(rates)
    rng = np.random.Generator(np.random.PCG64(args.seed + 77))
    t0 = time.time()
    srv = dfpr.Server(int(args.heap_gb * (1 << 30)), lanes=args.lanes)
    graphs = []  # (gid, n, m, batches)
    total_req = per_run * runs
    owners = rng.integers(0, sum(c for _, c in mix), size=total_req)  # graph of every request, uniform
    fracs = np.exp(rng.uniform(np.log(1e-6), np.log(1e-3), size=total_req))
    k = 0
    m_res = 0
    for sc, cnt in mix:
        for _ in range(cnt):
            n, s, d = W.rmat_graph(sc, 16, seed=args.seed * 131 + k)
            mine = np.nonzero(owners == k)[0]
            ch = chained_batches(n, s, d, fracs[mine], len(mine), seed=args.seed * 7 + k)
            g = dfpr.Graph.from_coo(n, torch.from_numpy(s).to("cuda"), torch.from_numpy(d).to("cuda"),
                                    row_slack=args.row_slack)
            m_res += g.m
            gid = srv.add_graph(g)
            graphs.append((gid, n, ch))
            k += 1
            del s, d
        log(f"  scale {sc}: {cnt} graphs resident ({time.time() - t0:.0f}s)")
    log(f"serving: {len(graphs)} graphs, {m_res} edges resident, heap {args.heap_gb:g} GiB, "
        f"{args.lanes} lanes, setup {time.time() - t0:.0f}s")
    cursor = [0] * len(graphs)
    order = list(owners)
    pos = [0]

    def run(rate, lanes):
        srv.set_active_lanes(lanes)
        gaps = rng.exponential(1.0 / rate, size=per_run)
        reqs = []
        for _ in range(per_run):
            gk = int(order[pos[0]])
            pos[0] += 1
            reqs.append((gk, graphs[gk][2][cursor[gk]]))
            cursor[gk] += 1
        tickets = [None] * per_run
        lat = [0.0] * per_run
        edges = [0] * per_run

        span = [0.0, 0.0]

        def submitter():
            t_start = time.perf_counter()
            due = 0.0
            for i, (gk, b) in enumerate(reqs):
                due += gaps[i]
                wait = t_start + due - time.perf_counter()
                if wait > 0:
                    time.sleep(wait)
                edges[i] = len(b[0]) + len(b[2])
                tickets[i] = srv.submit(graphs[gk][0], *b)
            span[0], span[1] = t_start, time.perf_counter()

        th = threading.Thread(target=submitter)
        t_begin = time.perf_counter()
        th.start()
        local = 0
        for i in range(per_run):
            while tickets[i] is None:
                time.sleep(0.0002)
            _, st, info, lat[i], _ = srv.wait(tickets[i])
            local += info["row_local"]
        t_end = time.perf_counter()
        th.join()
        el = t_end - t_begin
        return {"rate_per_s": rate, "arrival_rate_actual": per_run / max(span[1] - span[0], 1e-9), "lanes": lanes,
                "requests": per_run, "p50_ms": pct(lat, 50),
                "p99_ms": pct(lat, 99), "mean_ms": float(np.mean(lat)), "updates_per_s": per_run / el,
                "batch_edges_per_s": sum(edges) / el, "elapsed_s": el, "row_local_applies": local}

    results = []
    for rate in rates:
        mixr = run(rate, args.lanes)
        fifo = run(rate, 1)
        log(f"rate {rate:g}/s: {args.lanes} lanes p50 {mixr['p50_ms']:.2f} p99 {mixr['p99_ms']:.2f} ms "
            f"{mixr['updates_per_s']:.0f} upd/s | FIFO p50 {fifo['p50_ms']:.2f} p99 {fifo['p99_ms']:.2f} ms "
            f"{fifo['updates_per_s']:.0f} upd/s")
        results.append({"rate_per_s": rate, "served": mixr, "fifo": fifo})
    st = srv.stats()
    srv.close()
    best = max(results, key=lambda r: r["served"]["updates_per_s"])
    res = {
        "metric": "serving DF-P: p50/p99 update latency and updates/s vs one-at-a-time FIFO",
        "value": best["served"]["updates_per_s"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": per_run,
        "warmup": 0,
        "ms_per_step": best["served"]["mean_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(graphs)} resident R-MAT graphs (edge factor 16, scales "
                               + ", ".join(f"{c}x{sc}" for sc, c in mix) + "), Poisson arrivals, graph uniform, "
                               "batch f log-uniform in [1e-6, 1e-3] of |E|, 80/20, DF-P per request",
                   "edges_resident": int(m_res), "lanes": args.lanes, "heap_gib": args.heap_gb,
                   "requests_per_rate": per_run, "parallelism": "1 GPU",
                   **({"row_slack": args.row_slack} if args.row_slack else {})},
        "by_rate": results,
        "server_stats": st,
    }
    print(json.dumps(res))


def bench_temporal(args):
    """The temporal stream: 2M vertices, a 40M-edge stream in time order, the
    first 36M as G0, then insertion-only batches of 40,000 edges in time order
    (repeats of present edges are no-ops).  DF-P, DF and ND are chained (each
    starts from its own previous result); Static starts cold on every graph.
    With the oracle leg, the GPU DF-P chain and the oracle's own DF-P chain are
    compared after every one of the first batches (drift, not a parity gate:
    the per-step gate with equal inputs is a test)."""
    import torch
    import paper_2401_15870_amd as dfpr
    import workloads as W

    dev = torch.device("cuda:0")
    n, total, k0, B = 2_000_000, 40_000_000, 36_000_000, 40_000
    t0 = time.time()
    src, dst = W.temporal_stream(n, total, seed=args.seed + 6)
    steps = min(args.steps, (len(src) - k0) // B)
    log(f"temporal: n={n} stream={len(src)} initial {k0}, {steps} batches of {B} ({time.time() - t0:.0f}s)")
    s0, d0 = torch.from_numpy(src[:k0]).to(dev), torch.from_numpy(dst[:k0]).to(dev)
    modes = ("dfp", "df", "nd")
    gs = {m: dfpr.Graph.from_coo(n, s0, d0, row_slack=args.row_slack) for m in modes + ("static",)}
    if args.fused_limit is not None:
        for g in gs.values():
            g.set_fused_limit(args.fused_limit)
    if args.bounds:
        bounds = [int(x) for x in args.bounds.split(",")]
        for m in modes + ("static",):
            gs[m].set_tuning(bounds)
    elif not args.no_autotune:
        bounds, _ = gs["dfp"].autotune()
        for m in modes + ("static",):
            gs[m].set_tuning(bounds)
    log(f"bin bounds {gs['dfp'].get_tuning()}")
    m0 = gs["dfp"].m
    r0, _ = gs["static"].update_ranks("static", None)
    ranks = {m: r0.clone() for m in modes}
    oracle_steps = 0 if args.no_cpu else min(10, steps)
    if oracle_steps:
        import oracle as O
        og = O.graph(n, src[:k0], dst[:k0])
        r_or = r0.cpu().numpy()
    ms = {m: [] for m in modes + ("static",)}
    it = {m: [] for m in modes + ("static",)}
    apply_ms, ever, drift, m_after, local_steps = [], [], [], 0, 0
    for b in range(steps):
        lo = k0 + b * B
        ins_s, ins_d = src[lo:lo + B], dst[lo:lo + B]
        dev_ins = (torch.from_numpy(ins_s).to(dev), torch.from_numpy(ins_d).to(dev))
        for m, g in gs.items():
            torch.cuda.synchronize()
            t = time.perf_counter()
            info = g.apply_batch([], [], *dev_ins)
            torch.cuda.synchronize()
            if m == "dfp":
                apply_ms.append((time.perf_counter() - t) * 1e3)
                m_after = info["m_after"]
                local_steps += info["row_local"]
        for m in modes + ("static",):
            torch.cuda.synchronize()
            t = time.perf_counter()
            if m == "static":
                _, st = gs[m].update_ranks("static", None)
            else:
                _, st = gs[m].update_ranks(m, ranks[m], out=ranks[m])
            ms[m].append((time.perf_counter() - t) * 1e3)
            it[m].append(st["iterations"])
            if m == "dfp":
                ever.append(st["ever_affected"])
                dfp_st = st
        if b < oracle_steps:
            og2, ob = O.apply(og, [], [], ins_s, ins_d)
            r_or = O.rank("dfp", og2, r_or, og, ob).ranks
            og = og2
            drift.append(float(np.abs(ranks["dfp"].cpu().numpy() - r_or).max()))
        if b % 10 == 0 or b + 1 == steps:
            log(f"batch {b}: apply {apply_ms[-1]:.2f} ms, dfp {ms['dfp'][-1]:.2f} ({it['dfp'][-1]} it), "
                f"df {ms['df'][-1]:.2f}, nd {ms['nd'][-1]:.2f}, static {ms['static'][-1]:.2f} ms; dfp "
                f"processed {dfp_st['vertex_updates']} pulled {dfp_st['edges_pulled']} "
                f"dense its {dfp_st['dense_iterations']} bins {dfp_st['bin_edges']}"
                + (f", drift vs oracle chain {drift[-1]:.2e}" if b < oracle_steps else ""))
    step = [a + r for a, r in zip(apply_ms, ms["dfp"])]
    res = {
        "metric": "DF-P update time & edges/s vs GPU Static at L\u221e err \u22641e-9; p50/p99 latency",
        "value": m_after / (pct(step, 50) * 1e-3), "unit": "edges/s", "n_gpus": 1, "steps": steps, "warmup": 0,
        "ms_per_step": float(np.mean(step)), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"temporal stream (preferential attachment, 10 % repeats), {n} vertices, "
                               f"first {k0} of {len(src)} edges as G0, chained insertion-only batches of {B} "
                               f"in time order; apply + DFP update per step",
                   "n": n, "m0": int(m0), "parallelism": "1 GPU",
                   **({"row_slack": args.row_slack, "row_local_steps": local_steps} if args.row_slack else {})},
        "p50_ms": pct(step, 50), "p99_ms": pct(step, 99), "apply_p50_ms": pct(apply_ms, 50),
        "update_p50_ms": {m: pct(ms[m], 50) for m in ms},
        "iterations_mean": {m: float(np.mean(it[m])) for m in it},
        "speedup_vs_static": {m: pct(ms["static"], 50) / pct(ms[m], 50) for m in modes},
        "ever_affected_mean": float(np.mean(ever)),
        "drift_vs_oracle_chain_linf": drift,
    }
    print(json.dumps(res))


def bench_sweep(args):
    """Frontier measures and tolerances (Section 4.2) on the temporal stream:
    mean DF-P update time and rank error (L1 against a reference Static run to
    500 iterations) per measure and tau_f (tau_p = tau_f), next to Static."""
    import torch
    import paper_2401_15870_amd as dfpr
    import workloads as W

    dev = torch.device("cuda:0")
    n, total = 2_000_000, 40_000_000
    t0 = time.time()
    src, dst = W.temporal_stream(n, total, seed=args.seed + 6)
    k0 = int(0.9 * len(src))
    B = max(1, int(round(args.sweep_batch * len(src))))
    log(f"sweep: temporal stream n={n} edges={len(src)} initial {k0}, batches of {B} ({time.time() - t0:.0f}s)")
    # (measure, tau_f, tau_p): the frontier measures with tau_p = tau_f (Section 4.2), then the
    # prune tolerance from tau_f down to tau_f / 1e4 at tau_f = 1e-6, 1e-7, 1e-8 (Section 4.3)
    configs = [("relative", tf, tf) for tf in (1e-1, 1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]
    configs += [(c, tf, tf) for c in ("absolute", "contrib") for tf in (1e-10, 1e-11, 1e-12, 1e-13, 1e-14, 1e-15)]
    if args.sweep_prune:
        configs += [("relative", tf, tf / 10 ** k) for tf in (1e-6, 1e-7, 1e-8) for k in range(0, 5)
                    if not (tf == 1e-6 and k == 0)]
    s0, d0 = torch.from_numpy(src[:k0]).to(dev), torch.from_numpy(dst[:k0]).to(dev)
    ref_g = dfpr.Graph.from_coo(n, s0, d0)
    static_g = dfpr.Graph.from_coo(n, s0, d0)
    handles = [dfpr.Graph.from_coo(n, s0, d0) for _ in configs]
    r_static, _ = static_g.update_ranks("static", None)
    ranks = [r_static.clone() for _ in configs]
    rows = {i: {"ms": [], "err": [], "it": [], "ever": []} for i in range(len(configs))}
    st_ms, st_err = [], []
    for b in range(args.steps):
        lo = k0 + b * B
        ins = (src[lo:lo + B], dst[lo:lo + B])
        for g in [ref_g, static_g] + handles:
            g.apply_batch([], [], *ins)
        r_ref, _ = ref_g.update_ranks("static", None, tol=1e-300, max_iters=500)
        rs, st = static_g.update_ranks("static", None, timing=True)
        st_ms.append(st["ms_total"])
        st_err.append(float((rs - r_ref).abs().sum()))
        for i, (crit, tf, tp) in enumerate(configs):
            r, st = handles[i].update_ranks("dfp", ranks[i], out=ranks[i], timing=True, criterion=crit,
                                            frontier_tol=tf, prune_tol=tp)
            rows[i]["ms"].append(st["ms_total"])
            rows[i]["err"].append(float((r - r_ref).abs().sum()))
            rows[i]["it"].append(st["iterations"])
            rows[i]["ever"].append(st["ever_affected"])
        log(f"batch {b}: static {st_ms[-1]:.2f} ms L1 {st_err[-1]:.2e}")
    static_mean = float(np.mean(st_ms))
    table = []
    for i, (crit, tf, tp) in enumerate(configs):
        ms = float(np.mean(rows[i]["ms"]))
        table.append({"criterion": crit, "tau_f": tf, "tau_p": tp, "ms_mean": ms, "speedup_vs_static": static_mean / ms,
                      "l1_error_mean": float(np.mean(rows[i]["err"])), "iterations_mean": float(np.mean(rows[i]["it"])),
                      "ever_affected_mean": float(np.mean(rows[i]["ever"]))})
        log(f"{crit:9s} tau_f {tf:7.0e} tau_p {tp:7.0e}: {ms:7.2f} ms  x{static_mean / ms:5.1f}  "
            f"L1 {table[-1]['l1_error_mean']:.2e}")
    res = {"metric": "DF-P update time and L1 rank error per frontier measure and tolerance",
           "value": max(t["speedup_vs_static"] for t in table if t["l1_error_mean"] <= float(np.mean(st_err))),
           "unit": "speedup vs Static at no more error than Static", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "higher_is_better": True, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"temporal stream, {n} vertices, {len(src)} edges, initial 90 %, insertion-only "
                                  f"batches of {B} edges ({args.sweep_batch:g} of the stream) in time order; DF-P; "
                                  "error = L1 against Static run to 500 iterations",
                      "parallelism": "1 GPU"},
           "static": {"ms_mean": static_mean, "l1_error_mean": float(np.mean(st_err))},
           "table": table}
    print(json.dumps(res))


def rocsparse_csrmv_ms(torch, crow, col, x, reps, timed):
    """rocSPARSE's FP64 CSR SpMV (analysis once, then y = A x with A's values
    all 1) on the caller's device tensors, through its C API."""
    import ctypes
    rs = ctypes.CDLL("librocsparse.so")
    n = x.shape[0]
    m = col.shape[0]
    vp = ctypes.c_void_p
    h, descr, info = vp(), vp(), vp()
    for fn, arg in ((rs.rocsparse_create_handle, h), (rs.rocsparse_create_mat_descr, descr),
                    (rs.rocsparse_create_mat_info, info)):
        if fn(ctypes.byref(arg)) != 0:
            raise RuntimeError(f"{fn.__name__} failed")
    try:
        stream = torch.cuda.current_stream().cuda_stream
        if rs.rocsparse_set_stream(h, vp(stream)) != 0:
            raise RuntimeError("rocsparse_set_stream failed")
        vals = torch.ones(m, dtype=torch.float64, device=x.device)
        y = torch.empty(n, dtype=torch.float64, device=x.device)
        none = 111  # rocsparse_operation_none
        ptr = lambda t: vp(t.data_ptr())
        st = rs.rocsparse_dcsrmv_analysis(h, none, ctypes.c_int32(n), ctypes.c_int32(n), ctypes.c_int32(m), descr,
                                          ptr(vals), ptr(crow), ptr(col), info)
        if st != 0:
            raise RuntimeError(f"rocsparse_dcsrmv_analysis status {st}")
        alpha, beta = ctypes.c_double(1.0), ctypes.c_double(0.0)

        def mv():
            s = rs.rocsparse_dcsrmv(h, none, ctypes.c_int32(n), ctypes.c_int32(n), ctypes.c_int32(m),
                                    ctypes.byref(alpha), descr, ptr(vals), ptr(crow), ptr(col), info, ptr(x),
                                    ctypes.byref(beta), ptr(y))
            if s != 0:
                raise RuntimeError(f"rocsparse_dcsrmv status {s}")
        ms = timed(mv, reps)
        torch.cuda.synchronize()
        return ms
    finally:
        torch.cuda.synchronize()
        rs.rocsparse_destroy_mat_info(info)
        rs.rocsparse_destroy_mat_descr(descr)
        rs.rocsparse_destroy_handle(h)


def bench_gather(args):
    """The Static pull launch against library routines that do its core work on
    the same graph in the library's internal vertex order: embedding_bag (sum
    of gathered contributions per in-row, no values), rocSPARSE's CSR SpMV
    (the same with an FP64 value per edge) and a plain gather of every
    in-edge's contribution.  None of them reads or writes the rank, flag or degree
    arrays the pull also handles, so they bound what the gathers alone cost."""
    import torch
    import paper_2401_15870_amd as dfpr
    import workloads as W
    dev = torch.device("cuda:0")
    t0 = time.time()
    if args.gather_graph == "temporal":  # G0 of the temporal workload
        n = 2_000_000
        src, dst = W.temporal_stream(n, 40_000_000, seed=args.seed + 6)
        src, dst = src[:36_000_000], dst[:36_000_000]
        desc = "temporal stream G0 (2M vertices, first 36M of 40M stream edges)"
    else:
        n, src, dst = W.rmat_graph(args.scale, args.edge_factor, seed=args.seed)
        desc = f"R-MAT scale {args.scale}, edge factor {args.edge_factor:g}"
    g = dfpr.Graph.from_coo(n, torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev))
    m = g.m
    log(f"gather: {desc}: n={n} m={m} ({time.time() - t0:.1f}s)")
    if not args.no_autotune:
        bounds, _ = g.autotune()
        log(f"autotune: bounds {bounds}")
    g.set_timing(True)
    r = torch.empty(n, dtype=torch.float64, device=dev)
    g.update_ranks("static", None, out=r)
    ms, launches = 0.0, 0
    for _ in range(max(1, args.static_runs)):
        _, st = g.update_ranks("static", None, out=r)
        ms += st["ms_pull"]
        launches += st["pull_launches"]
    lib_ms = ms / launches
    # the in-CSR in the library's internal order (decreasing in-degree, ties by id)
    off, idx = g.export(in_csr=True)
    off_t = torch.from_numpy(off.astype(np.int64)).to(dev)
    idx_t = torch.from_numpy(idx).to(dev).long()
    g.close()
    deg = off_t[1:] - off_t[:-1]
    key = (int(deg.max()) - deg) * n + torch.arange(n, device=dev)
    order = torch.sort(key).indices
    perm = torch.empty(n, dtype=torch.int64, device=dev)
    perm[order] = torch.arange(n, device=dev)
    rows = torch.repeat_interleave(torch.arange(n, device=dev), deg)
    ekey = perm[rows] * n + perm[idx_t]
    del rows, idx_t, key
    ekey = torch.sort(ekey).values
    col = (ekey % n).to(torch.int32)
    crow = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    crow[1:] = torch.cumsum(torch.bincount(ekey // n, minlength=n), 0)
    del ekey
    contrib = torch.rand(n, dtype=torch.float64, device=dev)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(3, args.steps)
    out = {"library_pull_static_ms": round(lib_ms, 4)}
    col64 = col.long()
    try:
        out["embedding_bag_sum_ms"] = round(timed(lambda: torch.nn.functional.embedding_bag(
            col64, contrib.view(n, 1), crow[:-1], mode="sum"), reps), 4)
    except Exception as e:  # reported, not fatal
        out["embedding_bag_sum_ms"] = f"failed: {type(e).__name__}: {e}"[:200]
    try:
        out["rocsparse_csrmv_ms"] = round(rocsparse_csrmv_ms(torch, crow.to(torch.int32), col, contrib, reps, timed), 4)
    except Exception as e:
        out["rocsparse_csrmv_ms"] = f"failed: {type(e).__name__}: {e}"[:200]
    try:
        out["index_select_ms"] = round(timed(lambda: torch.index_select(contrib, 0, col64), reps), 4)
    except Exception as e:
        out["index_select_ms"] = f"failed: {type(e).__name__}: {e}"[:200]
    out["copy_index_stream_ms"] = round(timed(lambda: col.clone(), reps), 4)
    log(json.dumps(out))
    gathers_per_s = m / (lib_ms * 1e-3)
    print(json.dumps({"metric": "Static pull launch vs library gather-sum routines on the same graph and order",
                      "value": round(gathers_per_s, 1), "unit": "in-edges/s (library pull)", "n_gpus": 1,
                      "steps": reps, "warmup": 1, "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"{desc}, in-CSR in decreasing in-degree order", "n": n, "m": m},
                      "times_ms": out}))


def summarize_main(args):
    """Print the profile summaries of a profiled run directory (see profiles/)."""
    d = args.summarize
    if os.path.isdir(os.path.join(d, "prof")):
        print(summarize_trace(os.path.join(d, "prof")))
    fd, wd = os.path.join(d, "pmc_FETCH_SIZE"), os.path.join(d, "pmc_WRITE_SIZE")
    if os.path.isdir(fd) and os.path.isdir(wd):
        c, total = summarize_counters(fd, wd, args.kernel)
        wkey = f"rmat{args.scale}_ef{args.edge_factor:g}_{args.mode}_f{args.frac:g}"
        print(f"workload: {wkey}")
        print(f"kernel: {args.kernel}")
        print(f"source_sha: {rank_source_sha()}")
        print(f"launches: {c['fetch']['launches']}")
        print(f"fetch_kib_per_launch: {c['fetch']['kib_per_launch']:.1f}")
        print(f"fetch_copy_factor: {c['fetch']['factor']:.3f}")
        print(f"write_kib_per_launch: {c['write']['kib_per_launch']:.1f}")
        print(f"write_copy_factor: {c['write']['factor']:.3f}")
        print(f"hbm_bytes_per_launch: {total:.0f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--edge-factor", type=float, default=16)
    ap.add_argument("--frac", type=float, default=1e-4)
    ap.add_argument("--mode", default="dfp", choices=["dfp", "df", "nd", "static"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--asynchronous", action="store_true",
                    help="DF/DF-P update ranks in place during iterations (not bit-reproducible)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle leg (R0 from GPU Static)")
    ap.add_argument("--dense-switch", type=float, default=None,
                    help="DF/DF-P: weight of the cost rule that picks the dense form for an iteration "
                         "(library default 1; inf: always dense, 0: never)")
    ap.add_argument("--row-slack", type=int, default=0,
                    help="free slots after every CSR row: small batches then merge into the rows they touch")
    ap.add_argument("--two-phase", action="store_true",
                    help="rmat/temporal: dense-form DF/DF-P iterations through the two-phase pull (dfpr_set_two_phase)")
    ap.add_argument("--fused-limit", type=int, default=None,
                    help="edge count up to which a rank update runs in one cooperative launch (library default)")
    ap.add_argument("--bounds", default=None, help="rmat, temporal: in-degree bin thresholds a,b,c,d,e instead of autotuning")
    ap.add_argument("--static-runs", type=int, default=3)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="finish with three 1 GiB device copies (counter calibration under a profiler)")
    ap.add_argument("--sweep-batch", type=float, default=1e-5, help="sweep: batch size as a fraction of the stream")
    ap.add_argument("--sweep-prune", action="store_true",
                    help="sweep: also vary tau_p from tau_f to tau_f/1e4 at tau_f = 1e-6, 1e-7, 1e-8")
    ap.add_argument("--workload", default="rmat", choices=["rmat", "batched", "serving", "sweep", "gather", "temporal"],
                    help="rmat: one large R-MAT graph (default); batched: many graphs in one batch handle; "
                         "serving: request loop over resident graphs; sweep: frontier measures and tolerances; "
                         "gather: the Static pull launch against library gather-sum routines; "
                         "temporal: chained insertion batches of the temporal stream")
    ap.add_argument("--rates", default="100,1000,10000", help="serving: Poisson arrival rates per second")
    ap.add_argument("--requests", type=int, default=1000, help="serving: requests per rate and server setting")
    ap.add_argument("--lanes", type=int, default=4, help="serving: request lanes")
    ap.add_argument("--heap-gb", type=float, default=64.0,
                    help="serving: device heap (GiB) for the graphs' CSRs and the requests' blocks")
    ap.add_argument("--serving-scale-offset", type=int, default=0,
                    help="serving: subtract this from every graph scale (smaller runs)")
    ap.add_argument("--graphs", type=int, default=512, help="batched: number of member graphs")
    ap.add_argument("--member-n", default="1e3,1e6", help="batched: range of member vertex counts (log-uniform)")
    ap.add_argument("--batch-loop", action="store_true",
                    help="batched: run the batch handle's updates with a launch per iteration (default: one launch)")
    ap.add_argument("--gather-graph", default="rmat", choices=["rmat", "temporal"],
                    help="gather: the R-MAT graph of --scale or the temporal workload's initial graph")
    ap.add_argument("--summarize", metavar="DIR",
                    help="print summaries of rocprofv3 output under DIR (prof/, pmc_FETCH_SIZE/, pmc_WRITE_SIZE/)")
    ap.add_argument("--kernel", default="dfpr::k_pull<3", help="kernel name prefix for --summarize counters")
    args = ap.parse_args()
    if args.summarize:
        summarize_main(args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs on one GPU only: sharding over several GPUs is "
                                   "described in the design notes, not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import paper_2401_15870_amd as dfpr
    import workloads as W

    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "serving":
        bench_serving(args)
        return
    if args.workload == "sweep":
        bench_sweep(args)
        return
    if args.workload == "gather":
        bench_gather(args)
        return
    if args.workload == "temporal":
        bench_temporal(args)
        return

    t0 = time.time()
    n, src, dst = W.rmat_graph(args.scale, args.edge_factor, seed=args.seed)
    log(f"graph: n={n} edges(no self-loops)={src.shape[0]} gen {time.time() - t0:.1f}s")
    batches = chained_batches(n, src, dst, args.frac, args.warmup + args.steps, seed=args.seed + 1000)
    log(f"batches: {len(batches)} x (del {len(batches[0][0])}, ins {len(batches[0][2])})")

    t0 = time.time()
    g = dfpr.Graph.from_coo(n, torch.from_numpy(src).to(dev), torch.from_numpy(dst).to(dev),
                            row_slack=args.row_slack)
    m0 = g.m
    if args.fused_limit is not None:
        g.set_fused_limit(args.fused_limit)
    if args.two_phase:
        g.set_two_phase(True)
    torch.cuda.synchronize()
    log(f"create: m={m0} row slack {args.row_slack} {time.time() - t0:.2f}s")
    dev_batches = [tuple(torch.from_numpy(a).to(dev) for a in b) for b in batches]
    if args.bounds:
        g.set_tuning([int(x) for x in args.bounds.split(",")])
        log(f"bounds: {g.get_tuning()}")
    elif not args.no_autotune:
        t0 = time.time()
        bounds, tune_ms = g.autotune()
        log(f"autotune: bounds {bounds} pull {tune_ms:.3f} ms ({time.time() - t0:.1f}s)")

    # ---- GPU Static (cold, from 1/N) on G0: the comparison baseline
    r_static = torch.empty(n, dtype=torch.float64, device=dev)
    static_ms, static_it = [], 0
    for _ in range(args.static_runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st = g.update_ranks("static", None, out=r_static)
        static_ms.append((time.perf_counter() - t) * 1e3)
        static_it = st["iterations"]
    log(f"GPU static: {np.median(static_ms):.2f} ms, {static_it} iterations")

    # ---- R0 and the oracle leg (first step on the CPU, same R0, same batch)
    cpu = None
    parity = None
    if not args.no_cpu:
        import oracle as O
        t0 = time.time()
        og = O.graph(n, src, dst)
        ref0 = O.rank("static", og)
        log(f"oracle setup: canonical + static ({ref0.iterations} it) {time.time() - t0:.1f}s "
            f"threads={O.num_threads()}")
        r0 = ref0.ranks
        ds, dd, is_, id_ = batches[0]
        t0 = time.perf_counter()
        og1, ob = O.apply(og, ds, dd, is_, id_)
        ref1 = O.rank(args.mode, og1, r0, og, ob)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": og1.m / t_cpu, "unit": "edges/s", "cores": O.num_threads(), "kind": "oracle",
               "sample": f"one step (apply + {args.mode.upper()} update) of the same scale-{args.scale} "
                         f"workload from the same R0 and batch; {t_cpu:.2f} s"}
        log(f"oracle step: {t_cpu:.2f}s it={ref1.iterations} ever={ref1.ever_affected}")
        del og
    else:
        r0 = r_static.cpu().numpy()
    r = torch.from_numpy(np.ascontiguousarray(r0)).to(dev)

    # ---- steps
    rank_kw = {} if args.dense_switch is None else {"dense_switch": args.dense_switch}
    g.set_timing(True)
    step_ms, apply_ms, rank_ms, iters, ever, row_local = [], [], [], [], [], []
    kern = {"pull": 0.0, "two_phase": 0.0, "commit": 0.0, "bin": 0.0, "mark": 0.0, "sort": 0.0,
            "rebuild_out": 0.0, "rebuild_in": 0.0}
    pull_launches, v_upd, e_pull, pull_bytes = 0, 0, 0, 0.0
    tp_passes, tp_bytes = 0, 0.0
    m_sum = 0
    total = args.warmup + args.steps
    torch.cuda.synchronize()
    t_begin = None
    for i in range(total):
        if i == args.warmup:
            torch.cuda.synchronize()
            t_begin = time.perf_counter()
        if i == total - 1:
            r_before_last = r.clone()  # for the ND comparison after the timed steps
        ta = time.perf_counter()
        info = g.apply_batch(*dev_batches[i])
        tb = time.perf_counter()
        r, st = g.update_ranks(args.mode, r, out=r, asynchronous=args.asynchronous, **rank_kw)
        tc = time.perf_counter()
        if i == 0 and cpu is not None:
            parity = float(np.abs(r.cpu().numpy() - ref1.ranks).max())
            log(f"full-size parity step 0: linf={parity:.3e} (gpu it={st['iterations']} "
                f"oracle it={ref1.iterations}; ever gpu={st['ever_affected']} oracle={ref1.ever_affected})")
            assert parity <= (1e-8 if args.asynchronous else 1e-9), f"full-size parity failed: {parity}"
        if i >= args.warmup:
            step_ms.append((tc - ta) * 1e3)
            apply_ms.append((tb - ta) * 1e3)
            rank_ms.append((tc - tb) * 1e3)
            iters.append(st["iterations"])
            ever.append(st["ever_affected"])
            m_sum += info["m_after"]
            row_local.append(info["row_local"])
            kern["pull"] += st["ms_pull"]
            pull_launches += st["pull_launches"]
            kern["two_phase"] += st["ms_two_phase"]
            tp_passes += st["two_phase_passes"]
            tp_bytes += st["two_phase_bytes"]
            v_upd += st["vertex_updates"]
            e_pull += st["edges_pulled"]
            pull_bytes += st["pull_bytes"]
            kern["commit"] += st["ms_commit"]
            kern["bin"] += st["ms_bin"]
            kern["mark"] += st["ms_mark"]
            kern["sort"] += info["ms_sort"]
            kern["rebuild_out"] += info["ms_rebuild"][0]
            kern["rebuild_in"] += info["ms_rebuild"][1]
            log(f"step {i - args.warmup}: {step_ms[-1]:.2f} ms (apply {apply_ms[-1]:.2f}"
                f"{' row-local' if info['row_local'] else ''}, rank {rank_ms[-1]:.2f}) "
                f"it={st['iterations']} dense={st['dense_iterations']} ever={st['ever_affected']} "
                f"upd={st['vertex_updates']} pulled={st['edges_pulled']} pull {st['ms_pull']:.2f} "
                f"{'two-phase %d x %.2f ' % (st['two_phase_passes'], st['ms_two_phase']) if st['two_phase_passes'] else ''}"
                f"commit {st['ms_commit']:.2f} bin {st['ms_bin']:.2f} mark {st['ms_mark']:.2f}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_begin
    K = args.steps
    # ---- GPU ND (Static warm-started from the ranks before the last batch, on
    # the graph after it): untimed by the step clock, reported beside Static
    nd_ms, nd_it = [], 0
    r_nd = torch.empty_like(r)
    for _ in range(args.static_runs):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, st_nd = g.update_ranks("nd", r_before_last, out=r_nd)
        nd_ms.append((time.perf_counter() - t) * 1e3)
        nd_it = st_nd["iterations"]
    log(f"GPU ND (warm, last batch): {np.median(nd_ms):.2f} ms, {nd_it} iterations")
    ms_per_step = elapsed * 1e3 / K
    m_mean = m_sum / K
    value = m_mean * K / elapsed

    # ---- roofline of the dominant kernel (largest summed time).  Pull bytes are
    # the library's per-launch algorithmic count (every gather counted).
    # rebuild: 4 B read + 4 B write per edge, plus old/new offset and touched flag per row
    rebuild_bytes = K * (8 * m_mean + 9 * n)
    cand = {"k_pull": (kern["pull"], pull_bytes, max(pull_launches, 1)),
            "k_rebuild": (kern["rebuild_out"] + kern["rebuild_in"], 2 * rebuild_bytes, 2 * K)}
    if tp_passes:  # one pass = k_tp_scatter + k_tp_accum + k_tp_finish
        cand["two_phase"] = (kern["two_phase"], tp_bytes, tp_passes)
    dom = max(cand, key=lambda k: cand[k][0])
    ms_k, bytes_k, nl = cand[dom]
    achieved = (bytes_k / nl) / (ms_k / nl * 1e-3) / 1e9 if ms_k > 0 else 0.0
    wkey = f"rmat{args.scale}_ef{args.edge_factor:g}_{args.mode}_f{args.frac:g}"
    traffic = measured_traffic(wkey) if dom == "k_pull" else None
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
            "launches": nl, "avg_launch_ms": round(ms_k / nl, 5), "bytes_per_launch": int(bytes_k / nl),
            "source_sha": rank_source_sha()}
    if dom == "k_pull" and ms_k > 0:
        # beside the algorithmic rate: the counter-measured rate (bytes fetched
        # into L2 from the memory side, Infinity Cache hits included) and the
        # rate of compulsory bytes (each contribution read once per launch)
        if traffic is not None:
            roof["traffic_gbs"] = round(traffic / (ms_k / nl * 1e-3) / 1e9, 1)
        compulsory = (pull_bytes - 8.0 * e_pull + 8.0 * min(float(n) * nl, float(e_pull))) / nl
        roof["compulsory_bytes_per_launch"] = int(compulsory)
        roof["compulsory_gbs"] = round(compulsory / (ms_k / nl * 1e-3) / 1e9, 1)
    roof["copy_gbs"] = round(device_copy_gbs(torch, dev), 1)  # streaming ceiling of this device

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"R-MAT scale {args.scale} (a,b,c=0.57,0.19,0.19), edge factor "
                               f"{args.edge_factor:g}, self-loops; chained 80/20 batches of "
                               f"{args.frac:g}*|E|; apply + {args.mode.upper()} update per step",
                   "n": n, "m": int(m0), "batch_edges": int(len(batches[0][0]) + len(batches[0][2])),
                   "mode": args.mode + (" asynchronous" if args.asynchronous else ""), "parallelism": "1 GPU",
                   "bin_bounds": g.get_tuning(),
                   **({"dense_switch": args.dense_switch} if args.dense_switch is not None else {}),
                   **({"two_phase": True} if args.two_phase else {}),
                   **({"row_slack": args.row_slack, "row_local_steps": int(sum(row_local))}
                      if args.row_slack else {})},
        "p50_ms": pct(step_ms, 50),
        "p99_ms": pct(step_ms, 99),
        "apply_p50_ms": pct(apply_ms, 50),
        "rank_p50_ms": pct(rank_ms, 50),
        "static_ms": float(np.median(static_ms)),
        "static_iterations": static_it,
        "nd_ms": float(np.median(nd_ms)),
        "nd_iterations": nd_it,
        "speedup_vs_static": float(np.median(static_ms)) / pct(step_ms, 50),
        "rank_speedup_vs_static": float(np.median(static_ms)) / pct(rank_ms, 50),
        "iterations_mean": float(np.mean(iters)),
        "ever_affected_mean": float(np.mean(ever)),
        "kernel_ms_per_step": {k: v / K for k, v in kern.items()},
        "full_size_parity_linf": parity,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res))
    if args.calib:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log("calibration: 3 copies of 1 GiB done")
    # destroy the graph while the HIP runtime is certainly intact (not from a
    # destructor at interpreter exit)
    g.close()
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()

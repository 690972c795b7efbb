"""Benchmark of the sketch hot path on one MI355X.

Headline workload (the largest configuration, one GPU): clusters64x2048_churn.
V = 2^20 vertices: 64 dense clusters of 2048 vertices (each G(2048, 0.5)),
a sparse G(n, 2n) on the other 917,504 vertices, 63 tree bridges plus 65
extra between clusters.  Setup phase: the sparse edges, the bridges and every
cluster's first-arrival spanning forest (1.97M updates).  Then 11 churn
rounds, each inserting every other cluster edge (66.9M) in a fresh random
order and deleting them all in another (1.34e8 updates per round), with 100
random bridges toggled every 1e5 updates (splits and merges of cluster
groups).  Sketch: C=20 columns x D=40 depths per vertex (13.4 GB resident in
HBM).  The whole stream is drawn before timing and held in HBM.

One step = one churn round through the whole path, in device batches of
the size and launch geometry the autotuner picks on a warm-up context:
classification, staged scatter into both endpoints' sketches, host forest
links/cuts, replacement rounds (component XOR-reduce + verify/sample) for
every broken tree.  K steps walk the stream's rounds in order; after the
last round a fresh context (set up untimed) starts from round 0 again.  The
setup phase of every context runs before the timed region.

Prints one JSON line: whole-job updates/s; the staged scatter's roofline
(bound by its integer ALU work: the method's one column hash per (update,
column) over the kernel time of every 8th launch taken with HIP events on
its stream, against the vector ALU peak; beside it the compulsory HBM bytes
= 8 B per update + 32 B per bucket the timed launches changed, counted by
the kernel, the HBM traffic of the committed rocprofv3 PMC profile and the
VALU issue rate of the committed SQ counter profile); the plain (atomic) kernel on the same workload; and the CPU oracle
timed on a bounded sample of the same stream (all host cores, and one).
--workload selects the extra measurements of the other workload recipes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# Vector ALU peak: 256 CUs x 4 SIMDs x 16 lanes at 2.4 GHz, i.e. one 64-lane
# wave instruction per CU per clock (full-rate 32-bit integer operations,
# multiplies included: measured at 0.85-0.89 per CU per clock).
VALU_PEAK_WAVE_INSTS = 256 * 2.4e9
ALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
# The method's own ALU work: one column hash per (update, column).  The
# SplitMix64 finalizer with the seed XOR on 64-bit words is 19 full-rate
# 32-bit lane operations on gfx950 (2 for the seed XOR, 3 per shift-XOR
# step, 4 per multiply by a 64-bit constant).
HASH_LANE_OPS = 19
CALIB_BYTES = 256 << 20  # plain copy used to scale the HBM byte counters
BATCH4 = 1_000_000
# the benchmark workload of the first build, kept as an extra measurement
V, C, D, SEED, BATCH = 16384, 14, 28, 0x5EED0001, 1_000_000
WORKLOAD = ("er16384_p0.3_del10: V=16384, G(V,0.3) inserts in random order then 10% random "
            "deletions (44,276,290 updates), 1,000,000-update batches, C=14 x D=28 buckets")


def algorithmic_bytes_per_update(C: int) -> int:
    # 8 B packed update read + 2 endpoints x C buckets x 16 B x (read + write)
    return 8 + 64 * C


def kernel_source_hash() -> str:
    """Hash of the kernel sources (kernels.hip and kernels.hpp): profile
    figures taken on other sources are not used."""
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2509_14433_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_entry(kernel: str, workload: str):
    """Per-launch figures of `kernel` on `workload` from the committed
    rocprofv3 PMC summary (profiles/pmc_traffic.json), or None when absent or
    taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        with open(path) as f:
            prof = json.load(f)
    except (OSError, ValueError):
        return None
    ent = prof.get(f"{kernel}@{workload}")
    if not ent or ent.get("kernel_sources_sha256_16") != kernel_source_hash():
        return None
    return ent


# Scatter launches timed with HIP events: every TIME_EVERY-th one (each
# event between two kernels idles the GPU for a few microseconds).
TIME_EVERY = 8


def run_path(cupk, torch, packed, sizes, steps, warmup, mode, time_kernels=TIME_EVERY,
             graph=False, tune=False):
    """Warm up, then time `steps` batches.  With `tune` (staged mode), the
    scatter geometry comes from the autotuner run on the stream's second
    batch by a context that has applied the first.  Returns (seconds,
    updates, ctr, geometry or None)."""
    offs = [0]
    for s in sizes:
        offs.append(offs[-1] + s)
    nb = len(sizes)
    geo = {}
    if tune and nb > 1:
        t = cupk.Context(V, C, D, SEED, scatter_mode=mode, max_batch=BATCH)
        t.apply_updates_device(packed[offs[0]:offs[1]])
        res = t.autotune(packed[offs[1]:offs[2]].contiguous())
        t.close()
        geo = {k: res[k] for k in ("tile_vertices", "lds_rows", "chunk_records", "tile_layout",
                                   "coarse_tiles")}

    def new_ctx():
        return cupk.Context(V, C, D, SEED, scatter_mode=mode, max_batch=BATCH,
                            time_kernels=time_kernels, use_graph=graph, **geo)

    # warmup on a throwaway context (code objects, buffers, clocks)
    w = new_ctx()
    for i in range(warmup):
        j = i % nb
        if j == 0 and i:
            w.close()
            w = new_ctx()
        w.apply_updates_device(packed[offs[j]:offs[j + 1]])
    w.sync()
    w.close()
    n_ctx = (steps + nb - 1) // nb
    ctxs = [new_ctx() for _ in range(max(1, n_ctx))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    for i in range(steps):
        j = i % nb
        ctxs[i // nb].apply_updates_device(packed[offs[j]:offs[j + 1]])
        total += sizes[j]
    for c in ctxs:
        c.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctr = {}
    for c in ctxs:
        for k, val in c.counters().items():
            ctr[k] = ctr.get(k, 0) + val
    for c in ctxs:
        c.close()
    return dt, total, ctr, (geo or None)


def cpu_baseline(u, v, d, sizes, budget_s=15.0):
    """The oracle (sketch + forest replay) on the first batches of the same
    stream, one host thread, until `budget_s` seconds have been spent."""
    import oracle
    sk = oracle.Sketch(V, C, D, SEED)
    fr = oracle.ForestReplay(sk)
    t0 = time.perf_counter()
    done, nbat, off = 0, 0, 0
    for s in sizes:
        fr.apply_batch(u[off:off + s], v[off:off + s], d[off:off + s])
        off += s
        done += s
        nbat += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {nbat} of {len(sizes)} batches ({done} updates) of the same "
                      f"stream: plain C sketch update + Python forest replay, one thread"}


def static_leg(cupk, torch, packed, sizes, reps=5):
    """Components of the final graph from the sketches alone (Boruvka over
    supernodes, App. A.1.1) on the resident sketch after the whole stream;
    the stream itself is applied untimed.  Reports the time per run and the
    vertex-slab rate of its first two rounds (every vertex slab is read once
    by the in-place samples of round 1 and once by round 2's reduction)
    against the HBM bound for those slabs."""
    ctx = cupk.Context(V, C, D, SEED, max_batch=BATCH)
    off = 0
    for s in sizes:
        ctx.apply_updates_device(packed[off:off + s])
        off += s
    ctx.sync()
    ctx.static_components()  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        _, _, info = ctx.static_components()
    dt = (time.perf_counter() - t0) / reps
    ctx.close()
    slab = C * D * 16
    return {"ms": round(dt * 1e3, 4), "rounds": info["rounds"],
            "components": info["n_components"], "sample_failed": info["sample_failed"],
            "vertex_slabs_per_s": round(2 * V / dt, 1),
            "hbm_bound_ms": round(2 * V * slab / (HBM_PEAK_GBS * 1e9) * 1e3, 5)}


def served_bursts_leg(cupk, torch, packed, u, v, d, window=4_000_000, closed=False):
    """The paper's query pattern through the serving loop (App. C.1): update
    periods of uniform length in [1000, 2000], each followed by a burst of
    period/9 connectivity queries on uniform random pairs.  The context
    first takes the stream up to the last `window` updates as device batches
    (untimed); the timed part is the window (the deletions, with forest-edge
    cuts), from host memory.  Latency is per query, submission to answer."""
    import numpy as np
    n = len(u)
    start = n - window
    ctx = cupk.Context(V, C, D, SEED, max_batch=BATCH)
    for off in range(0, start, BATCH):
        ctx.apply_updates_device(packed[off:min(start, off + BATCH)])
    ctx.sync()
    ctx.serve_start(max_batch=1 << 16, mem_budget_bytes=16 * 2000 * 8)
    rng = np.random.default_rng(23)
    tickets = []
    i = start
    nq = 0
    t0 = time.perf_counter()
    while i < n:
        period = int(rng.integers(1000, 2001))
        e = min(n, i + period)
        ctx.submit_updates(u[i:e], v[i:e], d[i:e])
        k = period // 9
        q = rng.integers(0, V, size=(2, k)).astype(np.uint32)
        t = ctx.submit_queries(q[0], q[1])[0]
        if closed:
            ctx.wait(t)        # one period in flight: latency without queueing
        else:
            tickets.append(t)
        nq += k
        i = e
    for t in tickets:
        ctx.wait(t)
    dt = time.perf_counter() - t0
    st = ctx.serve_stats()
    ctx.serve_stop()
    ctx.close()
    return {"value": round(window / dt, 1), "unit": "updates/s",
            "queries_per_s": round(nq / dt, 1), "queries": st["queries"],
            "query_p50_us": round(st["query_p50_us"], 1),
            "query_p99_us": round(st["query_p99_us"], 1),
            "query_max_us": round(st["query_max_us"], 1), "batches": st["batches"],
            "setup": f"last {window} updates (the deletions) in periods of U[1000, 2000] "
                     "updates, each followed by a burst of period/9 queries, host-memory input, "
                     + ("one period in flight (closed loop)" if closed else
                        "submitted as fast as admission allows (16 periods of budget)")}


def served_leg(cupk, u, v, d, rho=100_000, inflight=4, max_batch=BATCH):
    """The same stream through the serving loop: update requests of `rho`
    updates, each followed by a Connected query on a random pair, pushed as
    fast as memory admission allows (a budget of `inflight` requests).
    Inputs come from host memory (PCIe included).  Returns updates/s and the
    query latency percentiles (submission to answer)."""
    import numpy as np
    ctx = cupk.Context(V, C, D, SEED, max_batch=max_batch)
    ctx.serve_start(max_batch=max_batch, mem_budget_bytes=inflight * rho * 8)
    rng = np.random.default_rng(11)
    n = len(u)
    qs = rng.integers(0, V, size=(n // rho + 2, 2))
    t0 = time.perf_counter()
    tickets = []
    for k, s in enumerate(range(0, n, rho)):
        tickets.append(ctx.submit_updates(u[s:s + rho], v[s:s + rho], d[s:s + rho]))
        tickets.append(ctx.submit_query(int(qs[k, 0]), int(qs[k, 1])))
    for t in tickets:
        ctx.wait(t)
    dt = time.perf_counter() - t0
    st = ctx.serve_stats()
    ctx.serve_stop()
    ctx.close()
    return {"value": round(n / dt, 1), "unit": "updates/s", "queries": st["queries"],
            "query_p50_us": round(st["query_p50_us"], 1),
            "query_p99_us": round(st["query_p99_us"], 1),
            "query_max_us": round(st["query_max_us"], 1), "batches": st["batches"],
            "admission_waits": st["admission_waits"],
            "setup": f"update requests of {rho} updates, a query after each, admission budget "
                     f"{inflight} requests ({inflight * rho * 8} B), host-memory input"}


def _time_batches(cupk, torch, ctxkw, packed, sizes, V_, C_, D_, S_, tune_sample=None):
    """One context over the whole stream in the given batches; returns
    (seconds, counters, tune result)."""
    ctx = cupk.Context(V_, C_, D_, S_, **ctxkw)
    tune = None
    if tune_sample is not None:
        tune = ctx.autotune(tune_sample)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    off = 0
    for sz in sizes:
        ctx.apply_updates_device(packed[off:off + sz])
        off += sz
    ctx.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctr = ctx.counters()
    ctx.close()
    return dt, ctr, tune


def workload_leg(args, cupk, torch, np, streamgen):
    """Full-size runs of the other workload recipes (extra measurements)."""
    name = args.workload
    out = {"metric": "edge updates/sec", "unit": "updates/s", "n_gpus": 1, "data": "synthetic",
           "dtype": "u64"}
    if name in ("rmat17", "fixed_forest"):
        i = {"rmat17": 2, "fixed_forest": 5}[name]
        cfg = streamgen.CONFIGS[i]
        print(f"bench: generating {cfg['name']}", file=sys.stderr, flush=True)
        Vw = cfg["V"]
        Cw = streamgen.ceil_log2(Vw)
        Dw = 2 * Cw
        if name == "rmat17":
            n = cfg["n"]
            packed = torch.empty(n, dtype=torch.int64, device="cuda")
            off = 0
            for u, v, d in streamgen.rmat_chunks(cfg["logV"], n, cfg["del_prob"], cfg["seed"]):
                m = len(u)
                packed[off:off + m].copy_(torch.from_numpy(cupk.pack_updates(u, v, d)
                                                           .view(np.int64)))
                off += m
                print(f"bench: generated {off} of {n}", file=sys.stderr, flush=True)
            sizes = streamgen.ragged_sizes(n, cfg["batch"][0], cfg["batch"][1], cfg["seed"])
        else:
            u, v, d = streamgen.config_stream(i)
            n = len(u)
            print(f"bench: generated {n} updates", file=sys.stderr, flush=True)
            sizes = streamgen.fixed_sizes(n, cfg["batch"])
            packed = torch.empty(n, dtype=torch.int64, device="cuda")
            step = 1 << 26
            for off in range(0, n, step):
                e = min(n, off + step)
                packed[off:e].copy_(torch.from_numpy(
                    cupk.pack_updates(u[off:e], v[off:e], d[off:e]).view(np.int64)))
            del u, v, d
        torch.cuda.synchronize()
        sample = packed[: min(n, 1 << 20)].contiguous()
        res = {}
        legs = [("plain_atomic", dict(scatter_mode=cupk.SCATTER_ATOMIC), False),
                ("staged_autotuned", dict(scatter_mode=cupk.SCATTER_STAGED), True),
                ("staged_autotuned_graph", dict(scatter_mode=cupk.SCATTER_STAGED,
                                                use_graph=True), True)]
        if name != "fixed_forest":
            # flagged runs walked one update at a time instead of contracted
            legs.append(("staged_autotuned_walk_plain", dict(scatter_mode=cupk.SCATTER_STAGED,
                                                             walk_plain=True), True))
        for label, kw, tune in legs:
            print(f"bench: {name} {label}", file=sys.stderr, flush=True)
            # kernel timers on every TIME_EVERY-th launch, as in the main
            # path: an event between two kernels idles the GPU for a few
            # microseconds, much of a 1M-update pass
            dt, ctr, tr = _time_batches(cupk, torch, dict(kw, max_batch=max(sizes),
                                                          time_kernels=TIME_EVERY),
                                        packed, sizes, Vw, Cw, Dw, cfg["S"],
                                        sample if tune else None)
            res[label] = {"value": round(n / dt, 1), "seconds": round(dt, 4),
                          "scatter_ms": round(ctr["scatter_ms"], 3),
                          "bin_ms": round(ctr["bin_ms"], 3), "links": ctr["links"],
                          "cuts": ctr["cuts"], "rounds": ctr["rounds"],
                          "sample_failed": ctr["sample_failed"],
                          "host_flags_ms": round(ctr["host_flags_ms"], 1),
                          "host_rounds_ms": round(ctr["host_rounds_ms"], 1),
                          "walks_contracted": ctr["walks_contracted"],
                          "walks_fallback": ctr["walks_fallback"],
                          # updates that changed the forest (the single-level
                          # analogue of the paper's isolated updates)
                          "structural_rate": round((ctr["links"] + ctr["cuts"]) / n, 7)}
            if tr:
                res[label]["tune"] = {k: tr[k] for k in ("tile_layout", "tile_vertices",
                                                         "lds_rows", "chunk_records",
                                                         "coarse_tiles", "batch_target")}
        out.update({"workload": cfg["name"], "updates": n, "batches": len(sizes), "V": Vw,
                    "C": Cw, "D": Dw, "results": res})
    elif name == "levels":
        # the multi-level hierarchy on the benchmark stream, and on the
        # fixed-forest stream, against the single-level path
        res = {}
        for i, label in ((1, "standard"), (5, "fixed_forest")):
            cfg = streamgen.CONFIGS[i]
            print(f"bench: generating {cfg['name']}", file=sys.stderr, flush=True)
            u, v, d = streamgen.config_stream(i)
            n = len(u)
            packed = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
            del u, v, d
            sizes = streamgen.fixed_sizes(n, cfg["batch"])
            Vw = cfg["V"]
            Cw = streamgen.ceil_log2(Vw)
            for lv in (True, False):
                print(f"bench: levels={lv} {label}", file=sys.stderr, flush=True)
                dt, ctr, _ = _time_batches(cupk, torch, dict(levels=lv, max_batch=cfg["batch"]),
                                           packed, sizes, Vw, Cw, 2 * Cw, cfg["S"])
                res[f"{label}/{'levels' if lv else 'single_level'}"] = {
                    "value": round(n / dt, 1), "seconds": round(dt, 4), "links": ctr["links"],
                    "cuts": ctr["cuts"], "level_passes": ctr["level_passes"],
                    "level_repairs": ctr["level_repairs"], "level_failed": ctr["level_failed"],
                    "top_rounds": ctr["rounds"], "sample_failed": ctr["sample_failed"],
                    "host_rounds_ms": round(ctr["host_rounds_ms"], 3)}
            del packed
            torch.cuda.synchronize()
        out.update({"workload": "levels mode on er16384_p0.3_del10 and "
                                "er16384_p0.3_fixedforest, 1,000,000-update batches",
                    "results": res})
    elif name == "exact_sweep":
        # throughput against batch (buffer) size with per-update semantics
        # (exact mode) and with batch semantics, over a window of 1,000,000
        # updates: the first deletions of the benchmark stream (standard
        # stream: many forest-edge deletions) and the first deletions of the
        # fixed-forest stream (no forest-edge deletion)
        windows = []
        for i, label in ((1, "standard"), (5, "fixed_forest")):
            cfg = streamgen.CONFIGS[i]
            print(f"bench: generating {cfg['name']}", file=sys.stderr, flush=True)
            u, v, d = streamgen.config_stream(i)
            start = int(np.argmax(d))          # first deletion
            win = 1_000_000
            packed = torch.from_numpy(cupk.pack_updates(u[:start + win], v[:start + win],
                                                        d[:start + win]).view(np.int64)).cuda()
            windows.append((label, cfg, packed, start, win))
            del u, v, d
        res = {}
        for label, cfg, packed, start, win in windows:
            Vw = cfg["V"]
            Cw = streamgen.ceil_log2(Vw)
            for exact in (True, False):
                for bsz in (100, 1000, 10_000, 100_000, 1_000_000):
                    ctx = cupk.Context(Vw, Cw, 2 * Cw, cfg["S"], max_batch=1_000_000,
                                       exact=exact)
                    for off in range(0, start, 1_000_000):
                        ctx.apply_updates_device(packed[off:min(start, off + 1_000_000)])
                    ctx.sync()
                    c0 = ctx.counters()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for off in range(start, start + win, bsz):
                        ctx.apply_updates_device(packed[off:min(start + win, off + bsz)])
                    ctx.sync()
                    dt = time.perf_counter() - t0
                    c1 = ctx.counters()
                    ctx.close()
                    key = f"{label}/{'exact' if exact else 'batch'}/{bsz}"
                    res[key] = {"value": round(win / dt, 1), "seconds": round(dt, 4),
                                "cuts": c1["cuts"] - c0["cuts"],
                                "reverts": c1["reverts"] - c0["reverts"],
                                "rounds": c1["rounds"] - c0["rounds"]}
                    print(f"bench: {key} {res[key]}", file=sys.stderr, flush=True)
        out.update({"workload": "exact-mode buffer sweep: 1,000,000-update windows at the "
                                "first deletion of er16384_p0.3_del10 and "
                                "er16384_p0.3_fixedforest", "results": res})
    elif name == "er65536_served":
        cfg = streamgen.CONFIGS[3]
        Vw = cfg["V"]
        Cw = streamgen.ceil_log2(Vw)
        Dw = 2 * Cw
        print("bench: generating the insert phase", file=sys.stderr, flush=True)
        g = streamgen.ForestTargetedDeletes(Vw, cfg["p"], cfg["del_frac"], cfg["forest_frac"],
                                            cfg["seed"], cfg["rho"])
        # record the stream: deletions pick forest edges of the library's own
        # forest (untimed), so a replay with the same chunk boundaries hits
        # current forest edges again
        rec = list(g.insert_chunks())
        ctx = cupk.Context(Vw, Cw, Dw, cfg["S"])
        for ch in rec:
            ctx.apply_updates(*ch)
        nfd = 0
        print("bench: recording forest-targeted deletions", file=sys.stderr, flush=True)
        while True:
            fe = ctx.forest_edges()
            ch = g.delete_chunk([e[0] for e in fe], [e[1] for e in fe])
            if ch is None:
                break
            fset = set(fe)
            nfd += sum((a, b) in fset for a, b in zip(ch[0].tolist(), ch[1].tolist()))
            ctx.apply_updates(*ch)
            rec.append(ch)
        ctx.close()
        n = sum(len(ch[0]) for ch in rec)
        rng = np.random.default_rng(17)
        qs = rng.integers(0, Vw, size=(len(rec), 2))
        res = {}
        for inflight in (1, 4):
            print(f"bench: served replay inflight={inflight}", file=sys.stderr, flush=True)
            ctx = cupk.Context(Vw, Cw, Dw, cfg["S"], max_batch=cfg["rho"])
            ctx.serve_start(max_batch=cfg["rho"], mem_budget_bytes=inflight * cfg["rho"] * 8)
            t0 = time.perf_counter()
            tickets = []
            for k, ch in enumerate(rec):
                tickets.append(ctx.submit_updates(*ch))
                tickets.append(ctx.submit_query(int(qs[k, 0]), int(qs[k, 1])))
            for t in tickets:
                ctx.wait(t)
            dt = time.perf_counter() - t0
            st = ctx.serve_stats()
            ctx.serve_stop()
            c2 = ctx.counters()
            ctx.close()
            res[f"served_inflight{inflight}"] = {
                "value": round(n / dt, 1), "query_p50_us": round(st["query_p50_us"], 1),
                "query_p99_us": round(st["query_p99_us"], 1), "queries": st["queries"],
                "batches": st["batches"], "cuts": c2["cuts"], "rounds": c2["rounds"]}
        out.update({"workload": cfg["name"], "updates": n, "forest_deletions": nfd,
                    "V": Vw, "C": Cw, "D": Dw, "rho": cfg["rho"], "results": res,
                    "input": "host memory (PCIe included)"})
    print(json.dumps(out), flush=True)


def er16384_leg(args, cupk, np, torch, streamgen):
    """The first build's benchmark line (extra measurement): V=16384,
    G(V,0.3) then 10% deletions, 1M-update batches; one step = one batch."""
    print("bench: generating stream", file=sys.stderr, flush=True)
    u, v, d = streamgen.config_stream(1)
    n = len(u)
    sizes = streamgen.fixed_sizes(n, BATCH)
    packed = torch.from_numpy(cupk.pack_updates(u, v, d).view(np.int64)).cuda()
    torch.cuda.synchronize()

    mode = cupk.SCATTER_STAGED if args.mode == "staged" else cupk.SCATTER_ATOMIC
    print("bench: timing main path", file=sys.stderr, flush=True)
    dt, total, ctr, geo = run_path(cupk, torch, packed, sizes, args.steps, args.warmup, mode,
                                   graph=bool(args.graph),
                                   tune=args.mode == "staged" and not args.no_tune)
    value = total / dt
    bpu = algorithmic_bytes_per_update(C)
    # the timed launches (every TIME_EVERY-th of the timed region)
    launches = max(1, ctr["timed_launches"])
    kname = "k_tile_scatter" if args.mode == "staged" else "k_scatter_atomic"
    avg_ms = ctr["scatter_ms"] / launches
    upd_per_launch = ctr["timed_updates"] / launches
    achieved = bpu * upd_per_launch / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": (profile_entry(kname, "er16384_p0.3_del10") or {}).get(
                    "hbm_bytes_per_launch"),
                "kernel": kname, "kernel_avg_ms": round(avg_ms, 5),
                "bin_avg_ms": round(ctr["bin_ms"] / launches, 5),
                "bytes_per_update": bpu,
                "updates_per_launch": round(upd_per_launch, 1),
                "timed_launches": ctr["timed_launches"],
                "timed_every": TIME_EVERY}
    out = {
        "metric": "edge updates/sec + % HBM roofline; p50/p99 connectivity-query latency",
        "value": round(value, 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "V": V, "C": C, "D": D, "batch": BATCH,
                   "scatter": args.mode, "graph": bool(args.graph), "parallelism": "single GPU",
                   "geometry": geo},
        "roofline": roofline,
        "counters": {k: (round(val, 3) if isinstance(val, float) else val)
                     for k, val in ctr.items()},
    }
    if not args.no_plain and args.mode == "staged":
        print("bench: timing plain path", file=sys.stderr, flush=True)
        pdt, ptot, pctr, _ = run_path(cupk, torch, packed, sizes, args.steps, args.warmup,
                                      cupk.SCATTER_ATOMIC)
        pl = max(1, pctr["timed_launches"])
        pavg = pctr["scatter_ms"] / pl
        pach = bpu * (pctr["timed_updates"] / pl) / (pavg * 1e-3) / 1e9
        out["plain"] = {"value": round(ptot / pdt, 1), "unit": "updates/s",
                        "ms_per_step": round(pdt * 1e3 / args.steps, 4),
                        "kernel": "k_scatter_atomic", "kernel_avg_ms": round(pavg, 5),
                        "achieved_GBs": round(pach, 1), "frac": round(pach / HBM_PEAK_GBS, 4)}
    if not args.no_static:
        print("bench: timing static components", file=sys.stderr, flush=True)
        out["static_components"] = static_leg(cupk, torch, packed, sizes)
    if not args.no_serve:
        print("bench: timing served path", file=sys.stderr, flush=True)
        out["served"] = served_leg(cupk, u, v, d)
        out["query_latency_us"] = {"p50": out["served"]["query_p50_us"],
                                   "p99": out["served"]["query_p99_us"]}
        print("bench: timing served path with query bursts", file=sys.stderr, flush=True)
        out["served_bursts"] = served_bursts_leg(cupk, torch, packed, u, v, d)
        out["served_bursts_closed_loop"] = served_bursts_leg(cupk, torch, packed, u, v, d,
                                                             closed=True)
    if not args.no_cpu:
        print("bench: timing CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(u, v, d, sizes)
    print(json.dumps(out), flush=True)




# ---------------------------------------------------------------------------
# Headline: clusters64x2048_churn
# ---------------------------------------------------------------------------
def clusters_phases_device(np, torch, streamgen, cfg):
    """The stream's phases (setup, round 0, ..., round R-1) as device int64
    tensors of packed updates."""
    phases = []
    t0 = time.perf_counter()
    for k, ph in enumerate(streamgen.clustered_phases(cfg)):
        phases.append(torch.from_numpy(ph.view(np.int64)).to("cuda"))
        print(f"bench: drew {'setup' if k == 0 else f'round {k - 1}'} ({len(ph)} updates), "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
        del ph
    torch.cuda.synchronize()
    return phases


def _apply_phase(ctx, ph, batch):
    n = ph.shape[0]
    for s in range(0, n, batch):
        ctx.apply_updates_device(ph[s:min(n, s + batch)])


def _ctr_delta(c1, c0):
    return {k: c1[k] - c0.get(k, 0) for k in c1}


def run_clusters(cupk, torch, phases, cfg, steps, warmup, batch, mode, tune,
                 time_kernels=TIME_EVERY, label="main", tune_sample=1 << 24, geometry=None,
                 keep_batch=False):
    """Time `steps` churn rounds (see the module docstring).  With `tune`,
    a warm-up context (setup phase, then 1M-update batches of round 0 so
    that it has measured its host time per batch) runs the autotuner on a
    sample of round 0, and the timed contexts use the tuned geometry and
    batch target instead of `batch`.  Returns (seconds, updates, counters
    of the timed rounds, tune result, batch used).  `geometry` (tile
    vertices, LDS rows, chunk records) fixes the launch configuration
    instead of tuning it; `keep_batch` keeps `batch` and takes only the
    tuned geometry."""
    Vc = cfg["V"]
    Cc = streamgen_ceil_log2(Vc)
    nr = len(phases) - 1
    tuned = {}
    geo = {}
    if geometry:
        geo = dict(zip(("tile_vertices", "lds_rows", "chunk_records", "tile_layout",
                        "coarse_tiles"), geometry))
        tune = False

    def new_ctx(bsz, timed=False):
        # timed contexts sample every k-th launch, k chosen so that the
        # timed rounds hold at least four timed launches
        k = time_kernels
        if timed and time_kernels:
            nb = steps * max(1, -(-int(phases[1].shape[0]) // bsz))
            k = max(1, min(time_kernels, nb // 4))
        ctx = cupk.Context(Vc, Cc, 2 * Cc, cfg["S"], scatter_mode=mode, max_batch=bsz,
                           time_kernels=k, **geo)
        _apply_phase(ctx, phases[0], bsz)
        ctx.sync()
        return ctx

    if tune or warmup:
        w = new_ctx(BATCH4)
        start = 0
        if tune:
            # host history at 1M batches, then the tuner on a sample of round 0
            start = min(phases[1].shape[0], 8 * BATCH4)
            _apply_phase(w, phases[1][:start], BATCH4)
            w.sync()
            sample = phases[1][start:start + min(tune_sample, phases[1].shape[0] - start)]
            tuned = w.autotune(sample.contiguous())
            geo = {"tile_vertices": tuned["tile_vertices"], "lds_rows": tuned["lds_rows"],
                   "chunk_records": tuned["chunk_records"], "tile_layout": tuned["tile_layout"],
                   "coarse_tiles": tuned["coarse_tiles"]}
            if not keep_batch:
                batch = tuned["batch_target"]
            print(f"bench: {label} tuned {geo} batch {batch} (host "
                  f"{tuned['host_ms_per_batch']:.2f} ms per batch)", file=sys.stderr, flush=True)
        for i in range(warmup):
            if i and i % nr == 0:
                w.close()
                w = new_ctx(batch)
            ph = phases[1 + i % nr]
            _apply_phase(w, ph[start:] if i == 0 else ph, batch)
            w.sync()
            print(f"bench: {label} warmup round {i % nr}", file=sys.stderr, flush=True)
        w.close()
    n_ctx = max(1, (steps + nr - 1) // nr)
    ctxs = [new_ctx(batch, timed=True) for _ in range(n_ctx)]
    c0 = [c.counters() for c in ctxs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    for i in range(steps):
        ph = phases[1 + i % nr]
        _apply_phase(ctxs[i // nr], ph, batch)
        total += ph.shape[0]
        if i % 4 == 3:
            print(f"bench: {label} round {i + 1} of {steps} queued, "
                  f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    for c in ctxs:
        c.sync()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctr = {}
    for c, a0 in zip(ctxs, c0):
        for k, val in _ctr_delta(c.counters(), a0).items():
            ctr[k] = ctr.get(k, 0) + val
    for c in ctxs:
        c.close()
    return dt, total, ctr, tuned, batch


def streamgen_ceil_log2(V):
    return max(1, int(math.ceil(math.log2(V))))


def host_cpu():
    """(logical CPUs this process may use, CPU model name)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    model = "unknown"
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    return n, model


def cpu_baseline_clusters(np, streamgen, phases_host_sample, cfg, budget_s=12.0):
    """The oracle's sketch update (hash + XOR into both endpoints, no forest)
    on a bounded sample of the same stream: every host core (each thread
    owns 256-vertex blocks dealt round-robin), then one thread."""
    import oracle
    Vc = cfg["V"]
    Cc = streamgen_ceil_log2(Vc)
    nthreads, model = host_cpu()
    u, v, _ = streamgen.unpack(phases_host_sample)
    out = {}
    for label, t in (("all_cores", nthreads), ("one_thread", 1)):
        sk = oracle.Sketch(Vc, Cc, 2 * Cc, cfg["S"])
        step = 1 << 22 if t > 1 else 1 << 19
        done, used = 0, t
        t0 = time.perf_counter()
        while done < len(u) and time.perf_counter() - t0 < budget_s:
            e = min(len(u), done + step)
            used = sk.apply_threads(u[done:e], v[done:e], t)
            done = e
        dt = time.perf_counter() - t0
        out[label] = {"value": round(done / dt, 1), "cores": used, "updates": done,
                      "seconds": round(dt, 2)}
        del sk
        print(f"bench: cpu baseline {label}: {out[label]}", file=sys.stderr, flush=True)
    a = out["all_cores"]
    return {"value": a["value"], "unit": "updates/s", "cores": a["cores"], "kind": "oracle",
            "cpu_model": model, "nproc": nthreads,
            "sample": f"the first {a['updates']} updates of the same stream (setup phase, then "
                      f"churn round 0): the oracle's sketch update (column hashes + XOR into "
                      f"both endpoints' buckets) on every core, each thread owning 256-vertex "
                      f"blocks dealt round-robin; "
                      f"forest work and stream generation excluded",
            "one_thread": out["one_thread"]}


def served_forest_targeted_leg(cupk, np, torch, streamgen, inflight=4):
    """er65536_p0.2_forestdel through the serving loop: G(65536, 0.2) inserts
    in random order (4.3e8), then 10% of them deleted, 30% of each deletion
    chunk on current forest edges, in chunks of rho = 1e5 updates with two
    connectivity queries after every chunk (a random pair and the endpoints
    of the last deleted forest edge).  The stream is first recorded by
    driving a context chunk by chunk (one device batch per chunk, timed:
    the direct path), then replayed from host memory through the serving
    loop, submitted as fast as the device-memory admission of `inflight`
    chunks allows; latency is per query, submission to answer."""
    cfg = streamgen.CONFIGS[3]
    Vw, rho = cfg["V"], cfg["rho"]
    Cw = streamgen_ceil_log2(Vw)
    t0 = time.perf_counter()
    gen = streamgen.ForestTargetedDeletes(Vw, cfg["p"], cfg["del_frac"], cfg["forest_frac"],
                                          cfg["seed"], rho)
    print(f"bench: forest-targeted stream: {gen.m} inserts drawn in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    rec = []
    last_forest = {}  # deletion chunk -> its last deleted forest edge
    ctx = cupk.Context(Vw, Cw, 2 * Cw, cfg["S"], max_batch=rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_upd = 0
    for ch in gen.insert_chunks_packed():
        ctx.apply_updates_device(torch.from_numpy(ch.view(np.int64)).to("cuda"))
        rec.append(ch)
        n_upd += len(ch)
    n_forest = 0
    while True:
        fu, fv = ctx.forest_edge_arrays()
        fkeys = fu.astype(np.uint64) * np.uint64(Vw) + fv
        ch = gen.delete_chunk_packed(fkeys)
        if ch is None:
            break
        ctx.apply_updates_device(torch.from_numpy(ch.view(np.int64)).to("cuda"))
        u, v, _ = streamgen.unpack(ch)
        hit = np.flatnonzero(np.isin(u.astype(np.uint64) * np.uint64(Vw) + v, fkeys))
        n_forest += len(hit)
        if len(hit):
            last_forest[len(rec)] = (int(u[hit[-1]]), int(v[hit[-1]]))
        rec.append(ch)
        n_upd += len(ch)
        if len(rec) % 100 == 0:
            print(f"bench: forest-targeted recorded {len(rec)} chunks", file=sys.stderr,
                  flush=True)
    ctx.sync()
    t_direct = time.perf_counter() - t0
    cd = ctx.counters()
    ctx.close()
    gen.close()
    print(f"bench: forest-targeted direct path {n_upd / t_direct:.3e} updates/s "
          f"({n_forest} forest-edge deletions, {cd['cuts']} cuts, {cd['rounds']} rounds)",
          file=sys.stderr, flush=True)
    # queries: a random pair and the endpoints of the last deleted forest edge
    rng = np.random.default_rng(17)
    qs = rng.integers(0, Vw, size=(len(rec), 2)).astype(np.uint32)
    ctx = cupk.Context(Vw, Cw, 2 * Cw, cfg["S"], max_batch=rho)
    ctx.serve_start(max_batch=rho, mem_budget_bytes=inflight * rho * 8)
    t0 = time.perf_counter()
    tickets = []
    last = (0, 1)
    for k, ch in enumerate(rec):
        u, v, d = streamgen.unpack(ch)
        tickets.append(ctx.submit_updates(u, v, d))
        tickets.append(ctx.submit_query(int(qs[k, 0]), int(qs[k, 1])))
        if d[0]:
            last = last_forest.get(k, last)
            tickets.append(ctx.submit_query(*last))
        if k % 500 == 0:
            print(f"bench: served chunk {k} of {len(rec)}", file=sys.stderr, flush=True)
    for t in tickets:
        ctx.wait(t)
    dt = time.perf_counter() - t0
    st = ctx.serve_stats()
    ctx.serve_stop()
    c2 = ctx.counters()
    ctx.close()
    return {"workload": cfg["name"], "value": round(n_upd / dt, 1), "unit": "updates/s",
            "updates": n_upd, "queries": st["queries"],
            "query_p50_us": round(st["query_p50_us"], 1),
            "query_p99_us": round(st["query_p99_us"], 1),
            "query_max_us": round(st["query_max_us"], 1), "batches": st["batches"],
            "admission_waits": st["admission_waits"], "cuts": c2["cuts"],
            "rounds": c2["rounds"], "sample_failed": c2["sample_failed"],
            "forest_edge_deletions": n_forest,
            "direct": {"value": round(n_upd / t_direct, 1), "unit": "updates/s",
                       "note": "the same chunks as device batches, one call per chunk, "
                               "forest edges read before every deletion chunk"},
            "setup": f"V={Vw}, C={Cw}, D={2 * Cw}; chunks of {rho} updates from host memory "
                     f"(PCIe included), a random-pair query after every chunk and the "
                     f"endpoints of the last deleted forest edge after every deletion chunk; "
                     f"admission budget "
                     f"{inflight} chunks of device ring ({inflight * rho * 8} B)"}


def clusters_main(args, cupk, np, torch, streamgen):
    cfg = streamgen.CONFIGS[4]
    Vc = cfg["V"]
    Cc = streamgen_ceil_log2(Vc)
    Dc = 2 * Cc
    batch = args.batch or BATCH4
    print("bench: drawing clusters64x2048_churn", file=sys.stderr, flush=True)
    phases = clusters_phases_device(np, torch, streamgen, cfg)
    nr = len(phases) - 1
    round_len = [int(p.shape[0]) for p in phases[1:]]
    mode = cupk.SCATTER_STAGED if args.mode == "staged" else cupk.SCATTER_ATOMIC
    print("bench: timing main path", file=sys.stderr, flush=True)
    geometry = tuple(int(x) for x in args.geometry.split(",")) if args.geometry else None
    dt, total, ctr, tuned, batch = run_clusters(cupk, torch, phases, cfg, args.steps, args.warmup,
                                                batch, mode, tune=not args.no_tune,
                                                geometry=geometry,
                                                tune_sample=args.tune_sample)
    value = total / dt
    kname = "k_tile_scatter" if args.mode == "staged" else "k_scatter_atomic"
    launches = max(1, ctr["timed_launches"])
    avg_ms = ctr["scatter_ms"] / launches
    upd_per_launch = ctr["timed_updates"] / launches
    prof = profile_entry(kname, cfg["name"])
    if args.mode == "staged":
        buckets = ctr["timed_buckets"] / launches
        comp = 8 * upd_per_launch + 32 * buckets
        comp_gbs = comp / (avg_ms * 1e-3) / 1e9
        alu_ops = HASH_LANE_OPS * Cc * upd_per_launch
        alu_t = alu_ops / (avg_ms * 1e-3) / 1e12
        alu_peak = ALU_PEAK_LANE_OPS / 1e12
        roof = {"bound": "alu", "achieved": round(alu_t, 2), "peak": round(alu_peak, 2),
                "unit": "Tops/s", "frac": round(alu_t / alu_peak, 4),
                "traffic": prof.get("hbm_bytes_per_launch") if prof else None,
                "kernel": kname, "kernel_avg_ms": round(avg_ms, 5),
                "basis": f"algorithmic ALU work per launch: one column hash per (update, "
                         f"column), {HASH_LANE_OPS} 32-bit lane operations each (the SplitMix64 "
                         f"finalizer with its seed XOR on gfx950), C = {Cc}; peak 256 CU x 64 "
                         f"lanes x 2.4 GHz",
                "alu_ops_per_launch": round(alu_ops),
                "hbm": {"achieved": round(comp_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(comp_gbs / HBM_PEAK_GBS, 4),
                        "basis": "compulsory bytes per launch: 8 B per update + 32 B (16 B "
                                 "read + 16 B written) per bucket the launch changed in HBM, "
                                 "counted by the kernel on the timed launches",
                        "compulsory_bytes_per_launch": round(comp),
                        "compulsory_bytes_per_update": round(comp / max(1.0, upd_per_launch),
                                                             1),
                        "buckets_changed_per_launch": round(buckets)},
                "updates_per_launch": round(upd_per_launch, 1),
                "timed_launches": ctr["timed_launches"],
                "bin_avg_ms": round(ctr["bin_ms"] / launches, 5),
                "algorithmic_GBs": round(algorithmic_bytes_per_update(Cc) * upd_per_launch /
                                         (avg_ms * 1e-3) / 1e9, 1),
                "algorithmic_basis": f"8 + 64*C = {algorithmic_bytes_per_update(Cc)} B per "
                                     "update (every bucket update a 16 B read + write); not a "
                                     "roofline fraction"}
        if prof:
            roof["hbm"]["traffic_frac"] = round(prof["hbm_bytes_per_launch"] /
                                                (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9), 4)
            if prof.get("valu_insts_per_launch"):
                vi = prof["valu_insts_per_launch"]
                roof["valu"] = {"insts_per_launch": vi,
                                "issue_frac": round(vi / (avg_ms * 1e-3) / VALU_PEAK_WAVE_INSTS,
                                                    4),
                                "peak": "256 CU x 2.4 GHz = 6.14e11 wave instructions/s (one "
                                        "64-lane instruction per CU per clock)"}
    else:
        bpu = algorithmic_bytes_per_update(Cc)
        achieved = bpu * upd_per_launch / (avg_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": prof.get("hbm_bytes_per_launch") if prof else None,
                "kernel": kname, "kernel_avg_ms": round(avg_ms, 5),
                "basis": f"8 + 64*C = {bpu} B per update (each bucket a device atomic XOR)"}
    timed_rounds = [i % nr for i in range(args.steps)]
    out = {
        "metric": "edge updates/sec + % HBM roofline; p50/p99 connectivity-query latency",
        "value": round(value, 1), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"clusters64x2048_churn: V=2^20, 64 clusters G(2048,0.5) + sparse "
                               f"G(917504, 2n), 128 bridges toggled 100 per 1e5 updates; one "
                               f"step = one churn round (insert then delete the "
                               f"{(round_len[0] - 1) // 2 // 1000 * 1000}+ non-forest cluster "
                               f"edges, ~{round_len[0] / 1e6:.0f}M updates) in {batch}-update "
                               f"device batches ("
                               + ("batched form: geometry and batch size from the autotuner" if
                                  tuned else "fixed batches") +
                               f"); timed rounds {timed_rounds} (a fresh context after round "
                               f"{nr - 1}); setup phase untimed",
                   "V": Vc, "C": Cc, "D": Dc, "batch": batch, "scatter": args.mode,
                   "updates_timed": total, "parallelism": "single GPU"},
        "roofline": roof,
        "counters": {k: (round(val, 3) if isinstance(val, float) else val)
                     for k, val in ctr.items()},
    }
    if geometry:
        out["config"]["geometry"] = dict(zip(("tile_vertices", "lds_rows", "chunk_records",
                                              "tile_layout", "coarse_tiles"), geometry))
    if tuned:
        out["config"]["tuned"] = {k: tuned[k] for k in ("tile_layout", "tile_vertices", "lds_rows",
                                                        "chunk_records", "coarse_tiles",
                                                        "batch_target",
                                                        "host_ms_per_batch", "batch_sizes",
                                                        "batch_ms")}
    if not args.no_plain and args.mode == "staged":
        psteps = max(1, min(args.steps, args.plain_steps))
        print("bench: timing staged kernel in fixed 1M batches", file=sys.stderr, flush=True)
        sdt, stot, sctr, stuned, _ = run_clusters(cupk, torch, phases, cfg, psteps, 0, BATCH4,
                                                  mode, tune=not args.no_tune,
                                                  label="staged_1M", keep_batch=True,
                                                  tune_sample=BATCH4)
        sl = max(1, sctr["timed_launches"])
        savg = sctr["scatter_ms"] / sl
        scomp = (8 * sctr["timed_updates"] + 32 * sctr["timed_buckets"]) / sl
        out["staged_1M"] = {"value": round(stot / sdt, 1), "unit": "updates/s", "steps": psteps,
                            "geometry": ({k: stuned[k] for k in ("tile_layout", "tile_vertices",
                                                                 "lds_rows", "chunk_records",
                                                                 "coarse_tiles")}
                                         if stuned else None),
                            "ms_per_step": round(sdt * 1e3 / psteps, 3), "batch": BATCH4,
                            "kernel_avg_ms": round(savg, 5),
                            "compulsory_bytes_per_launch": round(scomp),
                            "frac": round(scomp / (savg * 1e-3) / (HBM_PEAK_GBS * 1e9), 4),
                            "host_flags_ms": round(sctr["host_flags_ms"], 1),
                            "host_rounds_ms": round(sctr["host_rounds_ms"], 1)}
        print("bench: timing plain path", file=sys.stderr, flush=True)
        pdt, ptot, pctr, _, _ = run_clusters(cupk, torch, phases, cfg, psteps, 0, BATCH4,
                                             cupk.SCATTER_ATOMIC, tune=False, label="plain")
        pl = max(1, pctr["timed_launches"])
        pavg = pctr["scatter_ms"] / pl
        bpu = algorithmic_bytes_per_update(Cc)
        pach = bpu * (pctr["timed_updates"] / pl) / (pavg * 1e-3) / 1e9
        out["plain"] = {"value": round(ptot / pdt, 1), "unit": "updates/s", "steps": psteps,
                        "batch": BATCH4,
                        "ms_per_step": round(pdt * 1e3 / psteps, 3),
                        "kernel": "k_scatter_atomic", "kernel_avg_ms": round(pavg, 5),
                        "achieved_GBs": round(pach, 1), "frac": round(pach / HBM_PEAK_GBS, 4),
                        "basis": f"8 + 64*C = {bpu} B per update",
                        "host_flags_ms": round(pctr["host_flags_ms"], 1),
                        "host_rounds_ms": round(pctr["host_rounds_ms"], 1)}
    sample = None
    if not args.no_cpu:
        sample = np.concatenate([phases[0].cpu().numpy(), phases[1][:60_000_000].cpu().numpy()]
                                ).view(np.uint64)
    del phases
    torch.cuda.empty_cache()
    if not args.no_serve:
        print("bench: timing served path (er65536 forest-targeted)", file=sys.stderr, flush=True)
        out["served"] = served_forest_targeted_leg(cupk, np, torch, streamgen)
        out["query_latency_us"] = {"p50": out["served"]["query_p50_us"],
                                   "p99": out["served"]["query_p99_us"],
                                   "workload": out["served"]["workload"]}
    if sample is not None:
        print("bench: timing CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_clusters(np, streamgen, sample, cfg)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=11,
                    help="churn rounds timed (headline); batches for --workload er16384")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=0, help="updates per device batch (headline)")
    ap.add_argument("--plain-steps", type=int, default=2,
                    help="churn rounds timed with the plain atomic kernel")
    ap.add_argument("--no-tune", action="store_true", help="headline: keep the default geometry")
    ap.add_argument("--tune-sample", type=int, default=1 << 26,
                    help="headline: updates in the autotuner's sample (the largest batch it "
                         "can choose), taken from churn round 0 after 8M updates of history")
    ap.add_argument("--geometry", default="",
                    help="headline: TILE_VERTICES,LDS_ROWS,CHUNK_RECORDS[,LAYOUT[,COARSE_TILES]] "
                         "instead of "
                         "the autotuner's (with --batch, a fixed launch configuration for "
                         "profiling; LAYOUT 1 = record, 2 = pair)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-kernel run")
    ap.add_argument("--no-serve", action="store_true", help="skip the served run")
    ap.add_argument("--no-static", action="store_true",
                    help="skip the static-components run on the final sketch")
    ap.add_argument("--mode", default="staged", choices=["staged", "atomic"])
    ap.add_argument("--graph", type=int, default=0,
                    help="1: replay each batch's device work as captured HIP graphs")
    ap.add_argument("--workload", default="clusters",
                    choices=["clusters", "er16384", "rmat17", "er65536_served", "fixed_forest",
                             "exact_sweep", "levels"],
                    help="clusters: the benchmark line; the others print extra full-size "
                         "measurements of the other workload recipes")
    ap.add_argument("--calib", action="store_true",
                    help="first run a plain 256 MiB device copy (4 times) as the reference "
                         "for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "sketch across GPUs is not implemented.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2509_14433_amd as cupk
    import streamgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.calib:
        src = torch.ones(CALIB_BYTES // 8, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(4):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "clusters":
        clusters_main(args, cupk, np, torch, streamgen)
    elif args.workload == "er16384":
        er16384_leg(args, cupk, np, torch, streamgen)
    else:
        workload_leg(args, cupk, torch, np, streamgen)


if __name__ == "__main__":
    main()

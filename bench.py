#!/usr/bin/env python3
"""Walk-throughput benchmark on one MI355X.

Default (the driver's ``--gpus 1 --steps K --warmup W``): the served mixed
workload on a resident weighted symmetric R-MAT graph with 2^26 vertices and
average degree 16 (about 1.06 G directed edges): requests of 1..4096 queries,
each DeepWalk (80 moves, ALIAS), PPR (stop 0.2 after each move, ALIAS) or
Node2Vec (p = 2, q = 0.5, 80 moves, O-REJ), served by continuous batching with
memory admission and graph-captured ticks.  W bursts of 4000 requests warm up;
the timed region serves K x 4000 requests submitted at once (a backlog, so the
server is saturated: admitted as slots and memory free up), and a "step" is
4000 of them.  Then p50/p99 request latency is measured with Poisson arrivals
at 0.7x the saturated request rate.

The four batch workloads (deepwalk-rmat12, ppr-rmat22, node2vec-rmat24,
metapath-rmat24) run first and are reported as nested objects, each with its
own roofline, schedules and oracle baseline.  Then ppr-rmat22 is walked from
a CSR file (the graph kept on disk, partitions loaded as the walks need
them) and reported as ``disk_graph``.  ``--workload NAME`` runs one workload
alone and prints its own line.

Metric: walk steps (moves) per second of walk time, graph and tables
resident in HBM (the paper's throughput: steps of all queries / execution
time, table preprocessing timed separately; Experimental Setup, "Metrics").
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
CSRC = "paper_2107_11983_amd/csrc/"
WALK_SOURCES = [CSRC + f for f in ("walk.hip", "walk_common.hpp", "trw_device.hpp", "trw_internal.hpp")]
SERVE_SOURCES = [CSRC + f for f in ("serve_kernel.hip", "serve_internal.hpp", "walk_common.hpp", "trw_device.hpp",
                                    "trw_internal.hpp")]
BATCH_WORKLOADS = ("deepwalk-rmat12", "ppr-rmat22", "node2vec-rmat24", "metapath-rmat24")
SERVED_WORKLOAD = "served-rmat26"
HOST_CPU_SHARE = 16    # host threads the oracle's parallel baseline may use

# Algorithmic bytes: per move the row range
# (two int32 row offsets) 8 B, the sampling entry the move needs and the path
# entry written 4 B; per query the source read, path[0], length and status.
ENTRY_BYTES = {"alias": 12, "naive": 4, "its": None, "orej": None}
PER_QUERY_BYTES = 4 + 4 + 4 + 1


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(tag, files):
    """HBM bytes per launch (total, read, written) from a committed rocprofv3 counter summary,
    if it was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"counters_{tag}.md")
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    kv = dict(re.findall(r"^- (\w+): ([0-9a-fA-F.e+]+)\s*$", text, flags=re.M))
    if kv.get("kernel_source_sha256_16") != source_hash(files):
        return None, "stale"
    try:
        return {"total": float(kv["traffic_bytes_per_launch"]), "read": float(kv.get("read_bytes_per_launch", "nan")),
                "write": float(kv.get("write_bytes_per_launch", "nan")),
                "l2_hit_rate": float(kv["l2_hit_rate"]) if "l2_hit_rate" in kv else None,
                "method": {"1": "request sizes (32/64/128-byte read requests, 32/64-byte writes)"}.get(
                    kv.get("traffic_method"), "FETCH_SIZE scaled by a 1 GiB copy")}, path
    except KeyError:
        return None, None


def gather_by_lines(roofline, measured, launch_ms, gather):
    """Every read request reaching HBM is a 128-byte line on gfx950: the counters' read bytes per
    launch / 128 over the launch time, against the measured random-gather ceiling (4 GiB and,
    when measured, 32 GiB of footprint)."""
    if measured.get("read") is None or measured["read"] != measured["read"]:
        return
    lines_s = measured["read"] / 128 / (launch_ms * 1e-3)
    roofline["read_lines_per_s"] = round(lines_s, 1)
    roofline["frac_of_dependent_gather_ceiling_by_lines"] = round(lines_s / gather["dependent_best_reads_per_s"], 4)
    if gather.get("large"):
        roofline["frac_of_32GiB_gather_ceiling_by_lines"] = round(
            lines_s / gather["large"]["dependent_reads_per_s"], 4)


def host_info():
    """CPU model and thread counts of this host (recorded with every oracle figure)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count()
    return {"cpu_model": model, "nproc": affinity, "os_cpu_count": os.cpu_count()}


class Ctx:
    """Modules and device handles shared by the benchmark's parts."""

    def __init__(self, np, torch, synth, trw, props, dev):
        self.np, self.torch, self.synth, self.trw = np, torch, synth, trw
        self.props, self.dev = props, dev
        self.gather = None

    def release(self):
        import gc
        gc.collect()
        self.torch.cuda.synchronize()
        self.torch.cuda.empty_cache()


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=None, help="one workload alone (default: the served headline, "
                                                     "with the batch workloads nested)")
    ap.add_argument("--sampler", default=None, help="default: the workload's first sampler")
    ap.add_argument("--mode", default="persistent", choices=["persistent", "per_step"])
    ap.add_argument("--wpl", type=int, default=0, help="walkers per lane (0 = library default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--coop", type=int, default=0, help="MetaPath row-scan wave threshold (0 = library default)")
    ap.add_argument("--nq", type=int, default=0, help="override the number of queries (throughput-vs-batch sweeps)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="headline only, without the nested batch workloads")
    ap.add_argument("--no-disk", action="store_true", help="without the walk from a graph file")
    ap.add_argument("--disk-only", action="store_true", help="only the walk from a graph file, as its own line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle CPU time (headline)")
    ap.add_argument("--cpu-seconds-nested", type=float, default=4.0, help="target oracle CPU time per nested workload")
    ap.add_argument("--serve-replay", type=int, default=4000,
                    help="requests per step: one block of the timed backlog, and one warm-up burst (a backlog "
                         "ends in partly filled ticks as its last requests drain; 4000 per step keeps that "
                         "tail a few percent of the timed span at 10 steps)")
    ap.add_argument("--serve-requests", type=int, default=10000, help="measured requests of the latency phase")
    ap.add_argument("--serve-scale", type=int, default=0, help="override the served graph's scale (tests)")
    ap.add_argument("--serve-slots-per-cu", type=int, default=4096)
    ap.add_argument("--serve-steps", type=int, default=64, help="moves per walker slot per tick")
    ap.add_argument("--serve-pipelined", type=int, default=1, help="0: serial ticks (read each tick before queueing the next)")
    ap.add_argument("--serve-max-requests", type=int, default=4096, help="requests the server holds admitted at once")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="offered requests/s (0: 0.7x the saturated rate)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for counter collection: a 1 GiB copy (calibration) then the timed kernel only")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this engine runs on one GPU; queries shard across GPUs with no exchange, "
              "since each walk reads only the shared graph, but only the 1-GPU figure is measured. Use --gpus 1.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2107_11983_amd as trw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    props = torch.cuda.get_device_properties(0)
    log(f"device {props.name} cus={props.multi_processor_count}")
    ctx = Ctx(np, torch, synth, trw, props, torch.device("cuda:0"))
    if not args.no_probe and not args.profile_pass:
        ctx.gather = probe_gather(trw, torch, ctx.dev, props.multi_processor_count)
        ctx.release()

    if args.disk_only:
        print(json.dumps(bench_disk(ctx)), flush=True)
        return
    if args.workload:
        wl = synth.WORKLOADS[args.workload]
        out = bench_served(args, wl, ctx) if wl.algo == "mixed" else bench_batch(args, wl, ctx)
        if out is not None:
            print(json.dumps(out), flush=True)
        return

    nested = {}
    if not args.no_batch and not args.profile_pass:
        for name in BATCH_WORKLOADS:
            t0 = time.time()
            nested[name] = bench_batch(args, synth.WORKLOADS[name], ctx, nested=True)
            ctx.release()
            log(f"nested {name}: {time.time() - t0:.1f}s")
    disk = None
    if not args.no_batch and not args.no_disk and not args.profile_pass:
        t0 = time.time()
        try:
            disk = bench_disk(ctx)
        except (OSError, trw.TrwError) as e:   # e.g. no room for the graph file: in the line, and go on
            disk = {"error": f"{type(e).__name__}: {e}"}
            log(f"disk graph: not measured ({disk['error']})")
        ctx.release()
        log(f"disk graph: {time.time() - t0:.1f}s")
    out = bench_served(args, synth.WORKLOADS[SERVED_WORKLOAD], ctx)
    if out is None:
        return
    out["batch_workloads"] = nested
    if disk is not None:
        out["disk_graph"] = disk
    print(json.dumps(out), flush=True)


def bench_disk(ctx):
    """ppr-rmat22's batch walked from a CSR file (trw_disk_walk): as one partition, and as
    17 vertex-range partitions with 16 resident at once, first with the file in the page
    cache (written just before), then with its pages dropped so the reads come from the
    disk; every output compared with the in-memory walk."""
    import tempfile

    np, torch, synth, trw = ctx.np, ctx.torch, ctx.synth, ctx.trw
    wl = synth.WORKLOADS["ppr-rmat22"]
    g = synth.make_graph(wl)
    path = os.path.join(tempfile.gettempdir(), f"trw_bench_{os.getpid()}.csr")
    try:
        trw.write_disk_graph(path, g.row_ptr.astype(np.int64), g.col, g.weight)
        file_bytes = os.path.getsize(path)
        src = torch.from_numpy(synth.make_sources(wl, g)).to(ctx.dev)
        nq = int(src.numel())
        p = trw.make_params("ppr", "alias", wl.max_len, wl.walk_seed, stop_q32=trw.stop_threshold(wl.stop_prob))
        G = trw.Graph(g.row_ptr, g.col, g.weight, device="cuda:0")
        alias = G.table("alias")
        bufs = trw.WalkBuffers(G, p, nq)
        trw.walk(G, alias, p, src, bufs=bufs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P2, L2, S2 = trw.walk(G, alias, p, src, bufs=bufs)
        torch.cuda.synchronize()
        mem_s = time.perf_counter() - t0
        moves = int(L2.to(torch.int64).sum())
        runs = []
        fd = os.open(path, os.O_RDONLY)
        os.fsync(fd)                                 # written back, so its pages can be dropped below
        os.close(fd)
        for parts, slots, cache in ((1, 1, "page"), (16, 16, "page"), (16, 16, "dropped")):
            D = trw.DiskGraph(path, 0 if parts == 1 else g.m // parts)
            D.walk(p, src[:1000], slots=D.parts)     # every partition's destinations checked once, untimed
            torch.cuda.synchronize()
            if cache == "dropped":                   # the file's pages out of the page cache: reads from the disk
                fd = os.open(path, os.O_RDONLY)
                os.posix_fadvise(fd, 0, 0, os.POSIX_FADV_DONTNEED)
                os.close(fd)
            t0 = time.perf_counter()
            P, L, S, st = D.walk(p, src, slots=slots)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            same = bool(torch.equal(L, L2) and torch.equal(S, S2))
            cols = torch.arange(wl.max_len + 1, device=P.device)[None, :]
            for a in range(0, nq, 1 << 20):
                if not same:
                    break
                b = min(nq, a + (1 << 20))
                keep = cols <= L[a:b, None]
                same = bool(torch.equal(torch.where(keep, P[a:b], 0), torch.where(keep, P2[a:b, :wl.max_len + 1], 0)))
            runs.append({"partitions": D.parts, "slots": slots, "file_cache": cache, "ms": round(dt * 1e3, 2),
                         "steps_per_s": moves / dt,
                         "vs_in_memory": (moves / dt) / (moves / mem_s), "same_as_in_memory": same,
                         "rounds": st["runs"], "loads": st["loads"], "bytes_read": st["bytes_read"],
                         "read_GBps": st["bytes_read"] / max(st["read_ns"], 1)})
            log(f"disk graph: {D.parts} partitions, {slots} resident, file pages {cache}: {dt * 1e3:.1f} ms, "
                f"{st['loads']} loads, "
                f"{st['bytes_read'] / 1e9:.2f} GB read, same as in memory: {same}")
            del P, L, S
            D.close()
        del P2, L2, S2, bufs
        G.close()
        return {"workload": "ppr-rmat22 from a CSR file", "algo": "ppr", "sampler": "alias", "nq": nq,
                "moves": moves, "file_bytes": file_bytes, "in_memory_ms": round(mem_s * 1e3, 3),
                "in_memory_steps_per_s": moves / mem_s, "runs": runs,
                "note": "file_cache page: the file was just written and its reads come from the page cache; "
                        "dropped: its pages were dropped first (fsync, posix_fadvise DONTNEED), so they come from "
                        "the disk; partitions' ALIAS tables built at each load"}
    finally:
        if os.path.exists(path):
            os.remove(path)


def bench_batch(args, wl, ctx, nested=False):
    """One batch workload: every query of the batch walked per launch.  Returns the bench line
    (nested=True: the same object without the driver's top-level keys, default launch knobs)."""
    np, torch, synth, trw = ctx.np, ctx.torch, ctx.synth, ctx.trw
    dev = ctx.dev
    stream = torch.cuda.current_stream()
    gather = ctx.gather
    sampler = (None if nested else args.sampler) or {"metapath": "its+index", "node2vec": "orej+eidx",
                               "deepwalk": "naive+adj"}.get(wl.algo, wl.samplers[0])
    t0 = time.time()
    g = synth.make_graph(wl)
    log(f"graph {wl.name}: n={g.n} m={g.m} dmax={int(g.degrees().max())} ({time.time() - t0:.1f}s)")
    src_np = synth.make_sources(wl, g, nq=(None if nested else args.nq) or None)
    nq = len(src_np)
    G = trw.Graph(g.row_ptr, g.col, g.weight, g.label, symmetric=wl.symmetric, device="cuda:0")
    nbad = G.validate()
    assert nbad == 0, f"graph failed validation ({nbad})"
    d_src = torch.from_numpy(src_np).to(dev)

    # Preprocessing: per-vertex tables, timed separately from the walk.
    tables, pre_ms = {}, {}
    variant_samplers = {"metapath": ("its+index", "its"), "node2vec": ("orej+eidx", "orej+adj", "orej"),
                        "deepwalk": ("naive+adj", "naive"), "ppr": ("alias", "its", "rej")}.get(wl.algo, wl.samplers)
    need = {sampler} if (args.no_variants or args.profile_pass) else set(variant_samplers) | {sampler}
    for s in sorted(need):
        if (s in ("alias", "its", "rej") and wl.algo in ("ppr", "deepwalk", "mixed")) or "+" in s:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if s == "its+index":
                tables[s] = G.label_index(wl.labels)
            elif s.endswith("+adj"):
                tables[s] = G.adjacency_index()
            elif s.endswith("+eidx"):
                tables[s] = G.edge_index()
            else:
                tables[s] = G.table(s)
            e1.record(stream)
            torch.cuda.synchronize()
            pre_ms[s] = e0.elapsed_time(e1)
            log(f"table {s}: {pre_ms[s]:.2f} ms")

    kw = {}
    if wl.algo == "ppr":
        kw["stop_q32"] = trw.stop_threshold(wl.stop_prob)
    if wl.algo == "node2vec":
        kw["n2v_thr_q16"] = trw.n2v_thresholds(*wl.n2v_pq)
    if wl.algo == "metapath":
        kw["schema"] = [int(x) for x in synth.make_schema(wl)]

    def params(s):
        return trw.make_params(wl.algo, s.split("+")[0], wl.max_len, wl.walk_seed, **kw)

    def tuning_for():
        t = {}
        if nested:
            return None
        if args.wpl:
            t["walkers_per_lane"] = args.wpl
        if args.blocks_per_cu:
            t["blocks_per_cu"] = args.blocks_per_cu
        if args.chunk:
            t["queue_chunk"] = args.chunk
        if args.coop:
            t["coop_degree"] = args.coop
        return trw.make_tuning(**t) if t else None

    def run(s, mode, warmup, steps, tuning=None):
        p = params(s)
        bufs = trw.WalkBuffers(G, p, nq, mode)
        table = tables.get(s)
        for _ in range(warmup):
            trw.walk(G, table, p, d_src, mode=mode, tuning=tuning, bufs=bufs)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t_start = time.perf_counter()
        for a, b in ev:
            a.record(stream)
            trw.walk(G, table, p, d_src, mode=mode, tuning=tuning, bufs=bufs)
            b.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_start
        per_launch_ms = [a.elapsed_time(b) for a, b in ev]
        lengths = bufs.lengths.to(torch.int64)
        moves = int(lengths.sum().item())
        st = bufs.status
        dead = int((st == trw.TRW_ST_DEAD_END).sum().item())
        badsrc = int((st == trw.TRW_ST_BAD_SOURCE).sum().item())
        del bufs
        return dict(moves=moves, dead_ends=dead, bad_sources=badsrc, wall_s=wall, per_launch_ms=per_launch_ms)

    mode_name = "persistent" if nested else args.mode
    mode = trw.MODES[mode_name]
    if args.profile_pass:
        # calibration: a plain device copy of exactly 1 GiB, then the walk
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        r = run(sampler, mode, 1, max(args.steps, 1), tuning_for())
        log(f"profile pass: {r['moves']} moves per launch, {np.mean(r['per_launch_ms']):.3f} ms per launch")
        return None

    log(f"main: {wl.algo}/{sampler} {mode_name} warmup={args.warmup} steps={args.steps}")
    main_r = run(sampler, mode, args.warmup, args.steps, tuning_for())
    ms_step = 1000.0 * main_r["wall_s"] / args.steps
    avg_launch_ms = float(np.mean(main_r["per_launch_ms"]))
    moves = main_r["moves"]
    value = moves * args.steps / main_r["wall_s"]
    log(f"main: {moves} moves per batch, {ms_step:.3f} ms per batch, {value:.4g} steps/s")

    # Roofline of the walk kernel: algorithmic bytes / kernel time.
    entry = ENTRY_BYTES.get(sampler)
    roofline = None
    valid_q = nq - main_r["bad_sources"]
    if entry is not None and wl.algo in ("ppr", "deepwalk"):
        row_reads = moves + main_r["dead_ends"]
        alg_bytes = 8 * row_reads + entry * moves + 4 * moves + PER_QUERY_BYTES * valid_q + 5 * main_r["bad_sources"]
        achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
        measured, src = read_traffic(f"{wl.name}_{sampler}_{mode_name}", WALK_SOURCES)
        traffic = measured["total"] if measured else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                    "kernel": f"k_walk_persistent<{wl.algo},{sampler}>" if mode_name == "persistent"
                    else f"k_bsp_step<{wl.algo},{sampler}>",
                    "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": round(avg_launch_ms, 4),
                    "random_reads_per_launch": row_reads + moves}
        # Random reads the kernel itself issues: the fused ALIAS entry (32 B,
        # candidates' row ranges included) is one read per move, plus the
        # source's row range; the plain sampler reads the slot and then the
        # next row's range.
        issued = {"alias": moves + valid_q, "naive": 2 * moves + valid_q}.get(sampler)
        if issued is not None:
            roofline["issued_random_reads_per_launch"] = issued
        if traffic is not None:
            roofline["traffic_frac_of_peak"] = round(traffic / (avg_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
            roofline["l2_hit_rate"] = measured.get("l2_hit_rate")
            if gather:
                gather_by_lines(roofline, measured, avg_launch_ms, gather)

    # Autotuned launch (the paper's pre-execution tuning): candidates timed on a
    # sample of the batch, then the whole batch timed with the winner.
    autotuned = None
    if not args.no_variants and not args.profile_pass:
        # the whole batch when one launch of it is short, else a sample of 2^20 queries
        n_tune = nq if avg_launch_ms < 50 else min(nq, 1 << 20)
        t0 = time.perf_counter()
        best, best_ms = trw.autotune(G, tables.get(sampler), params(sampler), d_src[:n_tune], mode=mode)
        tune_s = time.perf_counter() - t0
        # the autotuner's first candidate is the library default for this walk and table
        default, _ = trw.autotune(G, tables.get(sampler), params(sampler), d_src[:64], mode=mode, budget=1)
        kept = best.as_dict() == default.as_dict()
        if kept:       # the default itself: the batch's own timing stands
            v, ms_b = value, ms_step
        else:
            r = run(sampler, mode, 1, args.steps, best)
            v, ms_b = r["moves"] * args.steps / r["wall_s"], 1000 * r["wall_s"] / args.steps
        autotuned = {"tuning": best.as_dict(), "default_kept": kept, "tuned_on_queries": n_tune,
                     "tune_s": round(tune_s, 3), "steps_per_s": round(v, 1), "ms_per_batch": round(ms_b, 4),
                     "vs_default": round(v / value, 4)}
        log(f"autotuned {best.as_dict()} ({'default kept' if kept else 'candidate'}): {v:.4g} steps/s "
            f"({v / value:.3f}x default), tuning {tune_s:.2f}s")

    # Other samplers / schedules of the same workload (same queries, same graph).
    variants = {}
    if not args.no_variants:
        for s in variant_samplers:
            for mname in ("persistent", "per_step"):
                if s == sampler and mname == mode_name:
                    continue
                if ((wl.algo in ("ppr", "deepwalk") and s in ("alias", "its", "rej")) or "+" in s) and s not in tables:
                    continue
                r = run(s, trw.MODES[mname], 1, 3)
                v = r["moves"] * 3 / r["wall_s"]
                variants[f"{s}/{mname}"] = {"steps_per_s": round(v, 1), "ms_per_batch": round(1000 * r["wall_s"] / 3, 3),
                                            "moves": r["moves"]}
                log(f"variant {s}/{mname}: {v:.4g} steps/s")
        if wl.algo in ("ppr", "deepwalk") and sampler.startswith("naive") and mode_name == "persistent":
            # the general persistent kernel on a graph the LDS path would take
            r = run(sampler, mode, 1, 3, trw.make_tuning(no_lds_graph=1))
            v = r["moves"] * 3 / r["wall_s"]
            variants[f"{sampler}/persistent/no_lds_graph"] = {"steps_per_s": round(v, 1),
                                                              "ms_per_batch": round(1000 * r["wall_s"] / 3, 3),
                                                              "moves": r["moves"]}
            log(f"variant {sampler}/persistent/no_lds_graph: {v:.4g} steps/s")

    # The PPR estimate on the batch's outputs: each query's end vertex counted
    # (Random Walk based Algorithms, PPR), then the 100 highest counts.
    ppr_est = None
    if wl.algo == "ppr" and not args.no_variants:
        p = params(sampler)
        bufs = trw.WalkBuffers(G, p, nq, mode)
        trw.walk(G, tables.get(sampler), p, d_src, mode=mode, bufs=bufs)
        counts = torch.zeros((1, g.n), dtype=torch.int32, device=dev)
        skipped = torch.zeros(1, dtype=torch.int64, device=dev)
        t_ec, t_tk = [], []
        for _ in range(5):
            counts.zero_()
            a, b, c = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            a.record(stream)
            trw.ppr_end_counts(G, bufs.paths, bufs.lengths, bufs.status, counts=counts, skipped=skipped)
            b.record(stream)
            ids, vals = trw.topk(counts[0], 100)
            c.record(stream)
            torch.cuda.synchronize()
            t_ec.append(a.elapsed_time(b))
            t_tk.append(b.elapsed_time(c))
        ppr_est = {"end_counts_ms": round(float(np.median(t_ec)), 4), "topk_ms": round(float(np.median(t_tk)), 4),
                   "k": 100, "queries": nq, "vertices": g.n,
                   "distinct_end_vertices": int((counts[0] != 0).sum().item()),
                   "top_count": int(vals[0].item()), "walk_ms": round(avg_launch_ms, 4)}
        del bufs
        # the counting walk: the same PPR walk counting end vertices, no paths written
        counts2 = torch.zeros_like(counts)
        t_cw = []
        for _ in range(5):
            counts2.zero_()
            a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            a.record(stream)
            trw.ppr_walk_counts(G, tables.get(sampler), p, d_src, counts=counts2)
            b.record(stream)
            torch.cuda.synchronize()
            t_cw.append(a.elapsed_time(b))
        same = bool(torch.equal(counts, counts2))
        # and with only the counts kept (no per-query lengths or status)
        t_cn = []
        for _ in range(5):
            counts2.zero_()
            a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            a.record(stream)
            trw.ppr_walk_counts(G, tables.get(sampler), p, d_src, counts=counts2, outputs=False)
            b.record(stream)
            torch.cuda.synchronize()
            t_cn.append(a.elapsed_time(b))
        same_n = bool(torch.equal(counts, counts2))
        ppr_est["counting_walk_ms"] = round(float(np.median(t_cw)), 4)
        ppr_est["counting_walk_steps_per_s"] = round(moves / (ppr_est["counting_walk_ms"] * 1e-3), 1)
        ppr_est["counting_walk_counts_equal"] = same
        ppr_est["counts_only_walk_ms"] = round(float(np.median(t_cn)), 4)
        ppr_est["counts_only_walk_counts_equal"] = same_n
        log(f"ppr estimate: end counts {ppr_est['end_counts_ms']} ms, top-100 {ppr_est['topk_ms']} ms; "
            f"counting walk {ppr_est['counting_walk_ms']} ms (counts equal: {same}); counts only "
            f"{ppr_est['counts_only_walk_ms']} ms (counts equal: {same_n})")
        del counts, counts2

    # Streamed output: the same batch in chunks, packed on the device and copied
    # by DMA into pinned host buffers while the next chunk walks (the chunk
    # function does nothing, so this is the PCIe-inclusive rate of the path).
    streamed = None
    if wl.algo == "ppr" and not args.no_variants:
        import ctypes
        p = params(sampler)
        chunk = 1 << 21
        dbytes, hbytes = ctypes.c_size_t(0), ctypes.c_size_t(0)
        trw.check(trw._abi.trw_walk_stream_bytes(G.handle, ctypes.byref(p), chunk, ctypes.byref(dbytes),
                                                 ctypes.byref(hbytes)))
        dkeep, dws = trw._aligned(int(dbytes.value), device=dev)
        hkeep, hbuf = trw._aligned(int(hbytes.value), pin=True)
        got = {"entries": 0}

        def _count(_u, cp):
            c = cp.contents
            got["entries"] += int(ctypes.cast(c.offsets, ctypes.POINTER(ctypes.c_uint64))[c.nq])
            return 0
        cb = trw._abi.TRW_CHUNK_FN(_count)
        walls = []
        for rep in range(3):
            got["entries"] = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            trw.check(trw._abi.trw_walk_stream(G.handle, tables[sampler].handle if sampler in tables else None,
                                               ctypes.byref(p), ctypes.c_void_p(d_src.data_ptr()), nq, 0, chunk, None,
                                               ctypes.c_void_p(dws.data_ptr()), dws.numel(),
                                               ctypes.c_void_p(hbuf.data_ptr()), hbuf.numel(), cb, None,
                                               ctypes.c_void_p(stream.cuda_stream)))
            walls.append(time.perf_counter() - t0)
        w = float(np.median(walls[1:]))
        streamed = {"chunk_queries": chunk, "ms_per_batch": round(1e3 * w, 3),
                    "steps_per_s_pcie_inclusive": round(moves / w, 1), "entries_to_host": got["entries"],
                    "bytes_to_host": got["entries"] * 4 + nq * 13}
        log(f"streamed to host: {streamed['ms_per_batch']} ms per batch, "
            f"{streamed['steps_per_s_pcie_inclusive']:.4g} steps/s PCIe-inclusive")
        del dkeep, dws, hkeep, hbuf

    # Graphs larger than HBM: the same batch with the CSR arrays and / or the
    # ALIAS table in pinned host memory, read in place over the host link.
    host_res = None
    if wl.algo == "ppr" and sampler == "alias" and not args.no_variants:
        p = params(sampler)
        ref = trw.WalkBuffers(G, p, nq, mode)
        trw.walk(G, tables[sampler], p, d_src, mode=mode, bufs=ref)
        t0 = time.perf_counter()
        Gh = trw.Graph(g.row_ptr, g.col, g.weight, placement="host")
        pin_s = time.perf_counter() - t0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        th = Gh.table(sampler)                       # built into host memory
        e1.record(stream)
        torch.cuda.synchronize()
        host_res = {"graph_pin_s": round(pin_s, 3), "table_build_into_host_ms": round(e0.elapsed_time(e1), 2)}
        th_d = G.table(sampler, placement="host")    # the device graph's table, in host memory
        td_h = Gh.table(sampler, placement="device")
        torch.cuda.synchronize()
        bufs = trw.WalkBuffers(G, p, nq, mode)
        for key, GG, tt in (("table_in_host", G, th_d), ("graph_and_table_in_host", Gh, th),
                            ("graph_in_host", Gh, td_h)):
            t_h = []
            for _ in range(3):
                a, b = (torch.cuda.Event(enable_timing=True) for _ in range(2))
                a.record(stream)
                trw.walk(GG, tt, p, d_src, mode=mode, bufs=bufs)
                b.record(stream)
                torch.cuda.synchronize()
                t_h.append(a.elapsed_time(b))
            same = bool(torch.equal(bufs.lengths, ref.lengths) and torch.equal(bufs.status, ref.status))
            ms_h = float(np.median(t_h))
            host_res[key] = {"ms_per_batch": round(ms_h, 3), "steps_per_s": round(moves / (ms_h * 1e-3), 1),
                             "lengths_status_equal": same}
            log(f"host memory, {key}: {ms_h:.2f} ms per batch, {moves / (ms_h * 1e-3):.4g} steps/s (equal: {same})")
        th_d.close()
        del bufs, ref, th, th_d, td_h
        Gh.close()

    # The same walk written as a walk program (the step-centric programming
    # model, compiled at run time): what the generic framework costs.
    if not args.no_variants and not args.profile_pass:
        prog_src, user, ptab = None, (), None
        base = sampler.split("+")[0]
        if wl.algo in ("ppr", "deepwalk") and base in ("naive", "alias", "its"):
            prog_src = trw.programs.ppr(base) if wl.algo == "ppr" else trw.programs.deepwalk(base)
            user = (kw.get("stop_q32", 0),)
            ptab = tables.get(sampler) if base != "naive" else None
        elif wl.algo == "node2vec":
            prog_src, user = trw.programs.NODE2VEC, tuple(kw["n2v_thr_q16"])
            ptab = tables.get("orej+eidx")
        elif wl.algo == "metapath":
            prog_src, user = trw.programs.METAPATH, (len(kw["schema"]),) + tuple(kw["schema"])
        if prog_src is not None:
            t0 = time.perf_counter()
            prog = trw.Program(prog_src)
            compile_s = time.perf_counter() - t0
            prog.walk(G, ptab, d_src, wl.max_len, wl.walk_seed, user=user)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                _, plen, _ = prog.walk(G, ptab, d_src, wl.max_len, wl.walk_seed, user=user)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            pm = int(plen.to(torch.int64).sum().item())
            variants["program"] = {"steps_per_s": round(pm * 3 / wall, 1), "ms_per_batch": round(1000 * wall / 3, 3),
                                   "moves": pm, "compile_s": round(compile_s, 2)}
            log(f"variant program: {pm * 3 / wall:.4g} steps/s (compiled in {compile_s:.2f}s)")
            prog.close()

    # Issued random reads against the device's measured random-gather ceiling.
    if roofline is not None and gather:
        acc_s = roofline.get("issued_random_reads_per_launch", roofline["random_reads_per_launch"]) / (
            avg_launch_ms * 1e-3)
        roofline["issued_random_reads_per_s"] = round(acc_s, 1)
        roofline["frac_of_dependent_gather_ceiling"] = round(acc_s / gather["dependent_best_reads_per_s"], 4)
        roofline["frac_of_independent_gather_ceiling"] = round(acc_s / gather["independent_best_reads_per_s"], 4)

    cpu = cpu_par = None
    if not args.no_cpu_baseline:
        cpu, cpu_par = cpu_baseline(g, wl, sampler, src_np, kw,
                                    args.cpu_seconds_nested if nested else args.cpu_seconds)

    # Node2Vec and MetaPath: a move's algorithmic bytes depend on its darts, the
    # adjacency test's probes (binary search in the previous row) and the labels
    # it scans, which the oracle counts.  Their rates per move on the oracle's
    # sample of this batch scale the batch's moves.  The label index replaces
    # the scan by two offsets and one destination, so a MetaPath walk through
    # it needs no counts.
    counts = cpu.get("oracle_counters") if cpu else None
    per_move, alg_from = None, None
    if wl.algo == "metapath" and sampler == "its+index":
        per_move, alg_from = 8 + 4 + 4, "label index: two offsets, one destination, the path entry"
    elif counts and wl.algo in ("node2vec", "metapath"):
        om = max(int(counts.get("moves", 0)), 1)
        if wl.algo == "node2vec":
            per_move = 8 + 4 * counts["orej_trials"] / om + 4 * counts["adjacency_probes"] / om + 4
        else:
            per_move = 8 + counts["label_reads"] / om + 4 + 4
        alg_from = "oracle counters on the cpu_baseline sample, per move"
    if roofline is None and per_move is not None:
        alg_bytes = int(per_move * moves + PER_QUERY_BYTES * valid_q + 5 * main_r["bad_sources"])
        achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
        measured, src = read_traffic(f"{wl.name}_{sampler}_{mode_name}", WALK_SOURCES)
        traffic = measured["total"] if measured else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                    "kernel": f"k_walk_persistent<{wl.algo},{sampler}>", "alg_bytes_per_launch": alg_bytes,
                    "avg_launch_ms": round(avg_launch_ms, 4), "alg_bytes_per_move": round(per_move, 3),
                    "alg_bytes_from": alg_from}
        if traffic is not None:
            roofline["traffic_frac_of_peak"] = round(traffic / (avg_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
            roofline["l2_hit_rate"] = measured.get("l2_hit_rate")
            if gather:
                gather_by_lines(roofline, measured, avg_launch_ms, gather)
        if wl.algo == "metapath" and sampler == "its+index":
            # one fused entry per move, plus the source's label offsets per query
            roofline["issued_random_reads_per_launch"] = moves + valid_q
            if gather:
                acc_s = (moves + valid_q) / (avg_launch_ms * 1e-3)
                roofline["issued_random_reads_per_s"] = round(acc_s, 1)
                roofline["frac_of_dependent_gather_ceiling"] = round(acc_s / gather["dependent_best_reads_per_s"], 4)
                roofline["frac_of_independent_gather_ceiling"] = round(
                    acc_s / gather["independent_best_reads_per_s"], 4)
        log(f"roofline ({wl.algo}): {per_move:.2f} algorithmic bytes per move, {achieved:.1f} GB/s")

    # MetaPath without the label index: the row scan's bytes priced by the oracle's label count per move
    if wl.algo == "metapath" and counts and "its/persistent" in variants:
        om = max(int(counts.get("moves", 0)), 1)
        per_scan = 8 + counts["label_reads"] / om + 4 + 4
        v = variants["its/persistent"]
        ab = int(per_scan * v["moves"] + PER_QUERY_BYTES * valid_q)
        ach = ab / (v["ms_per_batch"] * 1e-3) / 1e9
        v["roofline"] = {"bound": "hbm", "achieved": round(ach, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBPS, 5), "alg_bytes_per_move": round(per_scan, 2),
                         "alg_bytes_per_launch": ab, "kernel": "k_walk_persistent<metapath,its>",
                         "alg_bytes_from": "oracle label reads per move on the cpu_baseline sample"}
        traffic, _ = read_traffic(f"{wl.name}_its_persistent", WALK_SOURCES)
        v["roofline"]["traffic"] = traffic["total"] if traffic else None
        log(f"metapath row scan: {per_scan:.1f} algorithmic bytes per move, {ach:.1f} GB/s")

    out = {
        "metric": "walk steps/sec + % HBM roofline (1 GPU); p50/p99 query latency served",
        "value": round(value, 1),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{wl.name}: {wl.algo} sampler={sampler} mode={mode_name}; R-MAT 2^{wl.scale} "
                               f"{'symmetric' if wl.symmetric else 'directed'} avg deg {wl.avg_degree}"
                               f"{', uint32 weights 1..255' if wl.weights else ''}"
                               f"{', ' + str(wl.labels) + ' labels' if wl.labels else ''}; {nq} queries, max {wl.max_len} moves"
                               f"{', stop prob ' + str(wl.stop_prob) if wl.algo == 'ppr' else ''}",
                   "n": g.n, "m": g.m, "nq": nq, "moves_per_batch": moves, "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_parallel": cpu_par,
        "preprocess_ms": {k: round(v, 3) for k, v in pre_ms.items()},
        "autotuned": autotuned,
        "variants": variants,
        "ppr_estimate": ppr_est,
        "streamed_to_host": streamed,
        "host_resident": host_res,
        "gather_ceiling": gather,
    }
    if nested:
        for k in ("metric", "unit", "n_gpus", "steps", "warmup", "higher_is_better", "scaling", "vs_baseline",
                  "data", "gather_ceiling"):
            out.pop(k)
        out["steps_per_s"] = out.pop("value")
        out["ms_per_batch"] = out.pop("ms_per_step")
        out["batches"] = {"timed": args.steps, "warmup": args.warmup}
    return out



def bench_served(args, wl, ctx):
    """Served mixed workload: requests of 1..4096 queries, each DeepWalk (80 moves, ALIAS), PPR
    (stop 0.2, ALIAS) or Node2Vec (p=2, q=0.5, 80 moves, O-REJ with the edge index), on a resident
    weighted symmetric R-MAT graph; continuous batching with memory admission and graph-captured
    ticks.  W bursts of `serve_replay` requests warm up; timed: K such blocks submitted at once as
    one backlog (saturation).  Then p50/p99 request latency at 0.7x the saturated request rate,
    with Poisson arrivals."""
    import ctypes
    from paper_2107_11983_amd import _abi
    np, torch, synth, trw = ctx.np, ctx.torch, ctx.synth, ctx.trw
    t0 = time.time()
    g = synth.make_graph(wl, scale=args.serve_scale or None)
    log(f"graph {wl.name}: n={g.n} m={g.m} dmax={int(g.degrees().max())} ({time.time() - t0:.1f}s)")
    G = trw.Graph(g.row_ptr, g.col, g.weight, symmetric=True, device="cuda:0")
    assert G.validate() == 0
    pre = {}
    for name, fn in (("alias", lambda: G.table("alias")), ("edge_index", lambda: G.edge_index())):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        tab = fn()
        e1.record()
        torch.cuda.synchronize()
        pre[name] = round(e0.elapsed_time(e1), 3)
        if name == "alias":
            alias = tab
        else:
            eidx = tab
    log(f"tables {pre}")
    if args.profile_pass:
        # calibration for the counter passes: a plain device copy of exactly 1 GiB
        a = torch.empty(1 << 30, dtype=torch.uint8, device=ctx.dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    R, W, K = args.serve_replay, max(args.warmup, 0), max(args.steps, 1)
    n_lat_warm, n_lat = (0, 0) if args.profile_pass else (500, args.serve_requests)
    N = (W + K) * R + n_lat_warm + n_lat
    sizes, kinds, offs, src_np = synth.served_requests(wl, N, g.n)
    d_src = torch.from_numpy(src_np).cuda()
    d_kind = torch.repeat_interleave(torch.from_numpy(kinds.astype(np.int8)), torch.from_numpy(sizes)).cuda()
    stop_q32 = trw.stop_threshold(wl.stop_prob)
    n2v_thr = trw.n2v_thresholds(*wl.n2v_pq)
    algo_p = [trw.make_params("deepwalk", "alias", 80, wl.walk_seed),
              trw.make_params("ppr", "alias", 256, wl.walk_seed, stop_q32=stop_q32),
              trw.make_params("node2vec", "orej", 80, wl.walk_seed, n2v_thr_q16=n2v_thr)]
    strides = np.array([88, 264, 88])
    # Requests in blocks of R: W warm-up bursts, the K timed blocks (served as one backlog),
    # then the latency run.
    replays = [(i * R, (i + 1) * R) for i in range(W + K)]
    if n_lat:
        replays.append(((W + K) * R, N))
    # Paths: every request of the timed backlog has rows of its own, so no two requests in
    # flight at once share any; past 64 GiB of rows (a long --steps) its blocks of R requests
    # wrap round, and requests that share rows are then 64 GiB of rows apart.  The warm-up
    # bursts (each drained before the next) and the latency run take rows from the start again.
    # Lengths and status: a place for every query, tallied after the timed region.
    entries = sizes * strides[kinds]
    blk = np.arange(N) // R
    cs = np.concatenate([[0], np.cumsum(entries)])
    within = cs[:-1] - cs[blk * R]
    n_blk = int(blk[-1]) + 1
    block_need = int(max(cs[min(b * R + R, N)] - cs[b * R] for b in range(n_blk)))
    cap = max(1, (64 << 30) // (4 * block_need))
    n_parts = min(max(K, n_blk - (W + K)), cap)
    part = np.where(blk < W, 0, np.where(blk < W + K, blk - W, blk - (W + K))) % n_parts
    poff_all = part * block_need + within
    d_paths = torch.empty(n_parts * block_need, dtype=torch.int32, device="cuda")
    d_len = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    d_st = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")

    def make_reqs(lo, hi):
        """trw_request array for requests [lo, hi)."""
        reqs = (_abi.trw_request * (hi - lo))()
        for j, i in enumerate(range(lo, hi)):
            r = reqs[j]
            r.params = algo_p[kinds[i]]
            r.nq = int(sizes[i])
            r.sources = ctypes.c_void_p(d_src.data_ptr() + 4 * int(offs[i]))
            r.qid_base = i << 32
            r.paths = ctypes.c_void_p(d_paths.data_ptr() + 4 * int(poff_all[i]))
            r.path_stride = int(strides[kinds[i]])
            r.lengths = ctypes.c_void_p(d_len.data_ptr() + 4 * int(offs[i]))
            r.status = ctypes.c_void_p(d_st.data_ptr() + int(offs[i]))
        return reqs

    req_arrays = [make_reqs(lo, hi) for lo, hi in replays]
    arrivals_zero = [(ctypes.c_uint64 * (hi - lo))() for lo, hi in replays]
    completions = [(_abi.trw_completion * (hi - lo))() for lo, hi in replays]
    backlog = (W * R, (W + K) * R)
    req_backlog = make_reqs(*backlog)
    arrivals_backlog = (ctypes.c_uint64 * (K * R))()
    comp_backlog = (_abi.trw_completion * (K * R))()

    torch.cuda.synchronize()
    slots = ctx.props.multi_processor_count * args.serve_slots_per_cu
    srv = trw.Server(G, alias, eidx, pool_bytes=8 << 30, max_slots=slots, max_requests=args.serve_max_requests,
                     steps_per_tick=args.serve_steps, pipelined=bool(args.serve_pipelined))

    def serve(n, reqs, arrivals, comps):
        """Serve n requests arriving at the given offsets (ns from the start); returns the wall
        time and the server's moves, ticks and tick device time over the run."""
        s0 = srv.stats()
        t = time.perf_counter()
        rc = _abi.trw_probe_serve_replay(srv.handle, n, reqs, arrivals, comps, 600_000)
        wall = time.perf_counter() - t
        s1 = srv.stats()
        assert rc == 0, f"replay failed: {rc} {_abi.trw_last_error()}"
        return wall, {k: s1[k] - s0[k] for k in ("moves", "ticks", "tick_device_ns")}

    def replay(ri, arrivals=None):
        """Serve block ri (requests arriving at the given offsets, default all at once)."""
        lo, hi = replays[ri]
        wall, d = serve(hi - lo, req_arrays[ri], arrivals_zero[ri] if arrivals is None else arrivals,
                        completions[ri])
        return completions[ri], wall, d

    for r in range(W):
        _, wall, d = replay(r)
        log(f"warm-up burst {r}: {R / wall:.0f} req/s, {d['moves'] / wall:.4g} steps/s")
    # Timed: the K blocks as one backlog, every request submitted at the start, so admission
    # always has a request waiting (saturation); one ramp at the start and one drain at the end.
    tick0 = srv.stats()["ticks"]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    _, d = serve(K * R, req_backlog, arrivals_backlog, comp_backlog)
    torch.cuda.synchronize()
    region = time.perf_counter() - t_start
    moves, ticks, tick_ns = d["moves"], d["ticks"], d["tick_device_ns"]
    value = moves / region
    assert all(comp_backlog[i].status == 0 for i in range(K * R))
    # per-kind moves, dead ends and queries of the timed backlog
    q_lo, q_hi = int(offs[backlog[0]]), int(offs[backlog[1]])
    kq = d_kind[q_lo:q_hi].to(torch.int64)
    L = d_len[q_lo:q_hi].to(torch.int64)
    dead = (d_st[q_lo:q_hi] == trw.TRW_ST_DEAD_END).to(torch.int64)
    per_kind = np.array([[int(torch.where(kq == k, L, 0).sum()), int(torch.where(kq == k, dead, 0).sum()),
                          int((kq == k).sum())] for k in range(3)])
    assert int(per_kind[:, 0].sum()) == moves, "moves counted by the server and by the lengths differ"
    sat_rps = K * R / region
    log(f"timed: a backlog of {K} x {R} requests, {region:.3f}s: {sat_rps:.0f} req/s, {value:.4g} steps/s; "
        f"{ticks} ticks (tick {tick0}..{tick0 + ticks - 1} of this server), {tick_ns / max(ticks, 1) / 1e6:.4f} ms "
        f"device time per tick")
    if args.profile_pass:
        srv.close()
        return None
    # The same K blocks again as bursts, each drained before the next is submitted: the server
    # ramps up and drains once per block (context for the backlog figure, not timed with it).
    burst_walls, burst_moves = [], 0
    for r in range(W, W + K):
        _, wall, d = replay(r)
        burst_walls.append(wall)
        burst_moves += d["moves"]
    assert burst_moves == moves
    bursts = {"req_per_s": round(K * R / sum(burst_walls), 1), "steps_per_s": round(burst_moves / sum(burst_walls), 1),
              "burst_req_per_s": [round(R / w, 1) for w in burst_walls]}
    log(f"the same blocks as {K} bursts of {R}: {bursts['req_per_s']:.0f} req/s, {bursts['steps_per_s']:.4g} steps/s")

    # Latency: Poisson arrivals at 0.7x the saturated request rate (or a fixed rate).
    rate = args.serve_rate or 0.7 * sat_rps
    lat_lo, lat_hi = replays[-1]
    u = synth.uniform_f64(lat_hi - lat_lo, wl.walk_seed ^ 0x9015)
    arrivals = np.cumsum(-np.log(u) / rate) * 1e9
    arrivals -= arrivals[0]
    comp, wall_l, d_l = replay(len(replays) - 1, (ctypes.c_uint64 * (lat_hi - lat_lo))(*[int(x) for x in arrivals]))
    assert all(comp[i].status == 0 for i in range(lat_hi - lat_lo))
    lat = np.array([(comp[i].t_done_ns - comp[i].t_submit_ns) / 1e6 for i in range(n_lat_warm, n_lat_warm + n_lat)])
    queue = np.array([(comp[i].t_admit_ns - comp[i].t_submit_ns) / 1e6 for i in range(n_lat_warm, n_lat_warm + n_lat)])
    span = (comp[n_lat_warm + n_lat - 1].t_done_ns - comp[n_lat_warm].t_submit_ns) / 1e9
    log(f"latency at {rate:.0f} req/s offered: p50 {np.percentile(lat, 50):.3f} ms, p99 {np.percentile(lat, 99):.3f} ms")
    st = srv.stats()
    srv.close()

    # The same queries through the batch walker, per kind: the persistent kernel and the plain
    # one-launch-per-step schedule, over every request of the timed backlog (each kind's
    # queries in one launch, the batch walker's best case).
    lo, hi = replays[W][0], replays[W + K - 1][1]
    batch = {}
    for k, name in enumerate(synth.SERVED_KINDS):
        idx = [i for i in range(lo, hi) if kinds[i] == k]
        if not idx:
            continue
        src_k = torch.from_numpy(np.concatenate([src_np[offs[i]:offs[i + 1]] for i in idx])).cuda()
        p = algo_p[k]
        table = alias if k < 2 else eidx
        for mname in ("persistent", "per_step"):
            mode = trw.MODES[mname]
            bufs = trw.WalkBuffers(G, p, int(src_k.numel()), mode)
            trw.walk(G, table, p, src_k, mode=mode, bufs=bufs)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(3):
                trw.walk(G, table, p, src_k, mode=mode, bufs=bufs)
            b.record()
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / 3
            mv = int(bufs.lengths.to(torch.int64).sum().item())
            batch.setdefault(mname, {})[name] = {"queries": int(src_k.numel()), "moves": mv, "ms": round(ms, 4)}
            del bufs
    for mname, d in batch.items():
        mv = sum(v["moves"] for v in d.values())
        ms = sum(v["ms"] for v in d.values())
        d["all"] = {"moves": mv, "ms": round(ms, 4), "steps_per_s": round(mv / (ms * 1e-3), 1)}
        log(f"same queries, batch {mname}: {mv / (ms * 1e-3):.4g} steps/s")
    served_replay_sps = moves / region

    # Oracle on the same requests' queries (1 thread, then the same sample over the host's threads).
    cpu = cpu_par = None
    if not args.no_cpu_baseline:
        cpu, cpu_par = cpu_baseline_served(g, wl, ctx, replays[W], sizes, kinds, offs, src_np, stop_q32, n2v_thr,
                                           args.cpu_seconds)

    # Roofline of the tick kernel over the timed region: algorithmic bytes of the moves made
    # (ALIAS moves as the paper's method reads them; Node2Vec's darts and binary-search probes
    # per move from the oracle's counts on its sample), per tick, over the ticks' device time.
    counts = (cpu or {}).get("oracle_counters", {}).get("node2vec")
    moves_k = per_kind[:, 0]
    dead_k = per_kind[:, 1]
    queries = int(per_kind[:, 2].sum())
    if counts and counts.get("moves"):
        om = counts["moves"]
        n2v_per_move = 8 + 4 * counts["orej_trials"] / om + 4 * counts["adjacency_probes"] / om + 4
        darts_per_move = counts["orej_trials"] / om
        n2v_from = "oracle counters on the cpu_baseline sample, per move"
    else:
        n2v_per_move, darts_per_move, n2v_from = None, None, None
    alias_per_move = 8 + ENTRY_BYTES["alias"] + 4
    roofline = None
    if ticks and n2v_per_move is not None:
        alg_bytes = (alias_per_move * (moves_k[0] + moves_k[1]) + n2v_per_move * moves_k[2] + 8 * dead_k.sum()
                     + PER_QUERY_BYTES * queries)
        dev_s = tick_ns * 1e-9
        achieved = alg_bytes / dev_s / 1e9
        measured, _ = read_traffic(f"{wl.name}_serve_tick", SERVE_SOURCES)
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": measured["total"] if measured else None,
                    "kernel": "k_serve_tick", "launches": ticks, "avg_launch_ms": round(tick_ns / ticks / 1e6, 4),
                    "alg_bytes_per_launch": int(alg_bytes / ticks),
                    "alg_bytes_per_move": {"deepwalk_alias": alias_per_move, "ppr_alias": alias_per_move,
                                           "node2vec_orej": round(n2v_per_move, 3)},
                    "alg_bytes_from": f"ALIAS: row range, threshold and two destination ids, path entry; "
                                      f"Node2Vec: {n2v_from}",
                    "moves_by_kind": {k: int(v) for k, v in zip(synth.SERVED_KINDS, moves_k)},
                    "device_time_s": round(dev_s, 4), "timed_region_s": round(region, 4),
                    "device_busy_frac": round(dev_s / region, 4)}
        if measured:
            roofline["traffic_frac_of_peak"] = round(measured["total"] / (tick_ns / ticks * 1e-9) / 1e9 /
                                                     HBM_PEAK_GBPS, 4)
            roofline["l2_hit_rate"] = measured.get("l2_hit_rate")
            roofline["traffic_method"] = measured.get("method")
            if ctx.gather:
                gather_by_lines(roofline, measured, tick_ns / ticks * 1e-6, ctx.gather)
        if ctx.gather:
            # one random read per ALIAS move (the fused 32-byte entry), per Node2Vec dart (its
            # 16-byte adjacency record) and per query (the source's row range); the edge-set
            # probes of Node2Vec's neighbourhood test come on top, so this is a lower bound
            reads = (moves_k[0] + moves_k[1]) + darts_per_move * moves_k[2] + queries
            rs = reads / dev_s
            roofline["issued_random_reads_lower_bound_per_launch"] = int(reads / ticks)
            roofline["issued_random_reads_per_s"] = round(rs, 1)
            roofline["frac_of_dependent_gather_ceiling"] = round(rs / ctx.gather["dependent_best_reads_per_s"], 4)
            if ctx.gather.get("large"):
                roofline["frac_of_32GiB_gather_ceiling"] = round(rs / ctx.gather["large"]["dependent_reads_per_s"], 4)
        log(f"roofline (serve tick): {achieved:.1f} GB/s algorithmic, frac {achieved / HBM_PEAK_GBPS:.4f}")

    out = {
        "metric": "walk steps/sec + % HBM roofline (1 GPU); p50/p99 query latency served",
        "value": round(value, 1), "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(1000 * region / K, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: served mix of DeepWalk-80 ALIAS / PPR-0.2 ALIAS / Node2Vec p=2 q=0.5 "
                               f"len 80 (O-REJ, edge index), requests of U{{1..4096}} queries; a step is {R} "
                               f"requests of a backlog of {K * R} submitted at once (continuous batching); "
                               f"latency at Poisson arrivals "
                               f"{'%.0f req/s' % args.serve_rate if args.serve_rate else '0.7x saturation'}; "
                               f"R-MAT 2^{int(np.log2(g.n))} symmetric avg deg {wl.avg_degree}, uint32 weights 1..255",
                   "n": g.n, "m": g.m, "requests_per_step": R, "queries_timed": queries, "moves_timed": moves,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_baseline_parallel": cpu_par,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "mean": round(float(lat.mean()), 3), "queue_p50": round(float(np.percentile(queue, 50)), 3),
                       "queue_p99": round(float(np.percentile(queue, 99)), 3), "requests": n_lat,
                       "warmup_requests": n_lat_warm},
        "offered_req_per_s": round(rate, 1), "achieved_req_per_s": round(n_lat / span, 1),
        "steps_per_s_at_offered": round(d_l["moves"] / wall_l, 1),
        "saturated": {"req_per_s": round(sat_rps, 1), "steps_per_s": round(value, 1), "backlog_requests": K * R,
                      "bursts": bursts},
        "same_queries_batch_walker": batch,
        "served_vs_batch": {"served_saturated_steps_per_s": round(served_replay_sps, 1),
                            "vs_persistent": round(served_replay_sps / batch["persistent"]["all"]["steps_per_s"], 4),
                            "vs_per_step": round(served_replay_sps / batch["per_step"]["all"]["steps_per_s"], 4)},
        "server": {"ticks": st["ticks"], "steps_per_tick": args.serve_steps, "slots": slots,
                   "pipelined": bool(args.serve_pipelined), "max_requests": args.serve_max_requests, "pool_bytes": st["pool_bytes"],
                   "timed_ticks": ticks, "first_timed_tick": tick0},
        "preprocess_ms": pre,
        "gather_ceiling": ctx.gather,
    }
    del G, alias, eidx, d_paths, d_len, d_st, d_src, d_kind, req_arrays, completions
    return out


def probe_gather(trw, torch, dev, cus):
    """Best random-read rate over occupancy / chains, 4 GiB buffer of 16-byte elements."""
    import ctypes
    from paper_2107_11983_amd import _abi
    nbytes = 4 << 30
    buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    sink = torch.zeros(4096, dtype=torch.uint8, device=dev)
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert _abi.trw_probe_fill(ctypes.c_void_p(buf.data_ptr()), nbytes, 7, s) == 0
    res = {"buffer_bytes": nbytes, "elem_bytes": 16, "runs": []}
    best = {0: 0.0, 1: 0.0}
    steps = 64
    for dep in (1, 0):
        for chains in (1, 2, 4):
            for bpc in (4, 8):
                grid = cus * bpc
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                args = (ctypes.c_void_p(buf.data_ptr()), nbytes, 16, chains, steps, dep, grid, 256,
                        ctypes.c_void_p(sink.data_ptr()), s)
                assert _abi.trw_probe_gather(*args) == 0
                a.record()
                assert _abi.trw_probe_gather(*args) == 0
                b.record()
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                reads = grid * 256 * chains * steps
                rate = reads / (ms * 1e-3)
                best[dep] = max(best[dep], rate)
                res["runs"].append({"dependent": dep, "chains": chains, "blocks_per_cu": bpc,
                                    "reads_per_s": round(rate, 1), "ms": round(ms, 3)})
    res["dependent_best_reads_per_s"] = round(best[1], 1)
    res["independent_best_reads_per_s"] = round(best[0], 1)
    # every random read reaching HBM is a whole 128-byte line (the request-size counters)
    res["dependent_best_GBps_at_128B"] = round(best[1] * 128 / 1e9, 1)
    res["independent_best_GBps_at_128B"] = round(best[0] * 128 / 1e9, 1)
    log(f"gather ceiling: dependent {best[1]:.4g} reads/s, independent {best[0]:.4g} reads/s")
    # the same reads spread over 32 GiB, the size of the largest tables here (the rate falls
    # slowly with the footprint: address translation misses more often)
    top = max((r for r in res["runs"] if r["dependent"] == 1), key=lambda r: r["reads_per_s"])
    big_bytes = 32 << 30
    try:
        big = torch.empty(big_bytes, dtype=torch.uint8, device=dev)
    except RuntimeError:
        big = None
    if big is not None:
        assert _abi.trw_probe_fill(ctypes.c_void_p(big.data_ptr()), big_bytes, 7, s) == 0
        grid = cus * top["blocks_per_cu"]
        args = (ctypes.c_void_p(big.data_ptr()), big_bytes, 16, top["chains"], steps, 1, grid, 256,
                ctypes.c_void_p(sink.data_ptr()), s)
        assert _abi.trw_probe_gather(*args) == 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        assert _abi.trw_probe_gather(*args) == 0
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        rate = grid * 256 * top["chains"] * steps / (ms * 1e-3)
        res["large"] = {"buffer_bytes": big_bytes, "chains": top["chains"], "blocks_per_cu": top["blocks_per_cu"],
                        "dependent_reads_per_s": round(rate, 1)}
        log(f"gather ceiling over 32 GiB: dependent {rate:.4g} reads/s")
        del big
        torch.cuda.empty_cache()
    # the write side: random 16 B stores, 64 B blocks and whole 128 B lines
    res["scatter"] = {}
    for eb in (16, 64, 128):
        grid = cus * 4
        steps_w = 16
        args = (ctypes.c_void_p(buf.data_ptr()), nbytes, eb, steps_w, grid, 256, s)
        assert _abi.trw_probe_scatter(*args) == 0
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        assert _abi.trw_probe_scatter(*args) == 0
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        n = grid * 256 * steps_w
        res["scatter"][str(eb)] = {"writes_per_s": round(n / (ms * 1e-3), 1), "GBps": round(n * eb / (ms * 1e6), 1),
                                   "ms": round(ms, 3)}
        log(f"scatter {eb} B: {n / (ms * 1e-3):.4g} writes/s, {n * eb / (ms * 1e6):.1f} GB/s")
    del buf
    return res


def cpu_baseline(g, wl, sampler, src_np, kw, target_s):
    """The oracle (single-threaded C) on a bounded prefix of the same queries: one thread, and
    the same sample sharded over the host's cores.  Returns (single, parallel)."""
    try:
        import oracle
        oracle._load()
    except Exception as e:  # the oracle is test infrastructure; the GPU number does not depend on it
        log(f"cpu baseline skipped: {e}")
        return None, None
    algo = oracle.ALGOS[wl.algo]
    smp = oracle.SAMPLERS[sampler.split("+")[0]]   # indexes change reads, not results
    tab = {}
    t0 = time.time()
    if algo in (oracle.DEEPWALK, oracle.PPR) and smp == oracle.ALIAS:
        t, a = oracle.alias_build(g.row_ptr, g.weight)
        tab = dict(thr=t, alias=a)
    elif algo in (oracle.DEEPWALK, oracle.PPR) and smp == oracle.ITS:
        tab = dict(prefix=oracle.its_build(g.row_ptr, g.weight))
    elif algo in (oracle.DEEPWALK, oracle.PPR) and smp == oracle.REJ:
        tab = dict(weight=g.weight, pmax=oracle.rej_build(g.row_ptr, g.weight))
    if algo == oracle.METAPATH:
        tab = dict(label=g.label)
    log(f"cpu baseline: oracle tables {time.time() - t0:.1f}s")
    p = oracle.WalkParams(algo, smp, wl.max_len, wl.walk_seed, stop_q32=kw.get("stop_q32", 0),
                          n2v_thr_q16=tuple(kw.get("n2v_thr_q16", (65536,) * 3)), schema=tuple(kw.get("schema", ())))
    # calibrate on a small prefix, then size the timed sample to ~target_s
    n0 = min(len(src_np), 20000)
    t0 = time.perf_counter()
    r = oracle.walk(g.row_ptr, g.col, p, src_np[:n0], **tab)
    dt = time.perf_counter() - t0
    per_q = max(dt / n0, 1e-9)
    nsamp = int(min(len(src_np), max(n0, target_s / per_q)))
    piece = max(1, (2 << 30) // (4 * (wl.max_len + 1)))          # host paths buffer <= 2 GiB per call
    moves, dt = 0, 0.0
    counters = {}
    for lo in range(0, nsamp, piece):
        t0 = time.perf_counter()
        r = oracle.walk(g.row_ptr, g.col, p, src_np[lo:min(nsamp, lo + piece)], qid_base=lo, **tab)
        dt += time.perf_counter() - t0
        moves += int(r.lengths.sum())
        for k, v in r.counters.items():
            counters[k] = counters.get(k, 0) + int(v)
        del r
    log(f"cpu baseline: {nsamp} queries, {moves} moves in {dt:.2f}s")
    info = host_info()
    single = {"value": round(moves / dt, 1), "unit": "steps/s", "cores": 1, "kind": "oracle",
              "sample": f"first {nsamp} of {len(src_np)} queries of the same batch ({moves} moves, {dt:.1f} s, "
                        f"single thread, tables prebuilt)", "oracle_counters": counters, **info}
    # The same sample sharded by query range over the host's cores (the
    # oracle unchanged; ctypes releases the interpreter lock during each call).
    import concurrent.futures
    workers = max(1, min(HOST_CPU_SHARE, info["nproc"] or 1))
    shard = max(1, min(-(-nsamp // workers), piece))
    ranges = [(lo, min(nsamp, lo + shard)) for lo in range(0, nsamp, shard)]

    def run_range(r):
        out = oracle.walk(g.row_ptr, g.col, p, src_np[r[0]:r[1]], qid_base=r[0], **tab)
        return int(out.lengths.sum())

    t0 = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        pmoves = sum(ex.map(run_range, ranges))
    pdt = time.perf_counter() - t0
    assert pmoves == moves
    log(f"cpu baseline, {workers} threads: {pmoves} moves in {pdt:.2f}s")
    parallel = {"value": round(pmoves / pdt, 1), "unit": "steps/s", "cores": workers, "kind": "oracle",
                "sample": f"the same {nsamp} queries in {len(ranges)} query ranges over {workers} threads "
                          f"({pdt:.1f} s)", **info}
    return single, parallel


def cpu_baseline_served(g, wl, ctx, replay, sizes, kinds, offs, src_np, stop_q32, n2v_thr, target_s):
    """The oracle (single-threaded C) on the requests of one timed replay, in submission order,
    until about target_s of walking: one thread, then the same requests spread over the host's
    threads.  Returns (single, parallel); single carries the oracle's counters per request kind."""
    import synth
    try:
        import oracle
        oracle._load()
    except Exception as e:  # the oracle is test infrastructure; the GPU number does not depend on it
        log(f"cpu baseline skipped: {e}")
        return None, None
    t0 = time.time()
    thr, al = oracle.alias_build(g.row_ptr, g.weight)
    log(f"cpu baseline: oracle ALIAS table {time.time() - t0:.1f}s")
    params = [oracle.WalkParams(oracle.DEEPWALK, oracle.ALIAS, 80, wl.walk_seed),
              oracle.WalkParams(oracle.PPR, oracle.ALIAS, 256, wl.walk_seed, stop_q32=stop_q32),
              oracle.WalkParams(oracle.NODE2VEC, oracle.OREJ, 80, wl.walk_seed, n2v_thr_q16=tuple(n2v_thr))]

    def run(i):
        k = int(kinds[i])
        kw = dict(thr=thr, alias=al) if k < 2 else {}
        r = oracle.walk(g.row_ptr, g.col, params[k], src_np[offs[i]:offs[i + 1]], qid_base=i << 32, **kw)
        return k, int(r.lengths.sum()), r.counters

    lo, hi = replay
    done, moves, dt = [], 0, 0.0
    counters = {name: {} for name in synth.SERVED_KINDS}
    for i in range(lo, hi):
        t = time.perf_counter()
        k, mv, c = run(i)
        dt += time.perf_counter() - t
        done.append(i)
        moves += mv
        for key, v in c.items():
            counters[synth.SERVED_KINDS[k]][key] = counters[synth.SERVED_KINDS[k]].get(key, 0) + int(v)
        if dt >= target_s:
            break
    nq = int(sum(sizes[i] for i in done))
    log(f"cpu baseline: {len(done)} requests, {nq} queries, {moves} moves in {dt:.2f}s")
    info = host_info()
    single = {"value": round(moves / dt, 1), "unit": "steps/s", "cores": 1, "kind": "oracle",
              "sample": f"the first {len(done)} requests ({nq} queries, {moves} moves) of the first timed replay, "
                        f"in submission order, one thread, ALIAS table prebuilt ({dt:.1f} s)",
              "oracle_counters": counters, **info}
    import concurrent.futures
    workers = max(1, min(HOST_CPU_SHARE, info["nproc"] or 1))
    t = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        pmoves = sum(mv for _, mv, _ in ex.map(run, done))
    pdt = time.perf_counter() - t
    assert pmoves == moves
    log(f"cpu baseline, {workers} threads: {pmoves} moves in {pdt:.2f}s")
    parallel = {"value": round(pmoves / pdt, 1), "unit": "steps/s", "cores": workers, "kind": "oracle",
                "sample": f"the same {len(done)} requests, one per task, over {workers} threads ({pdt:.1f} s)", **info}
    del thr, al
    return single, parallel


if __name__ == "__main__":
    main()

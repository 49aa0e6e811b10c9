#!/usr/bin/env python3
"""Walk-throughput benchmark on one MI355X.

Default workload: PPR walks (stop probability 0.2 after each move, at most 256
moves) from 10^7 uniformly random sources on a weighted directed R-MAT graph
with 2^22 vertices and average degree 32 (uint32 weights in [1, 255]),
sampled with the integer ALIAS table, one persistent launch per batch.  A
"step" of this benchmark is one batch: all 10^7 queries walked to completion.

Metric: walk steps (moves) per second of walk time, graph and tables resident
in HBM (the paper's throughput: steps of all queries / execution time, table
preprocessing timed separately; Experimental Setup, "Metrics").

Printed: one JSON line with the throughput, a roofline object for the walk
kernel, the oracle's single-core throughput on a bounded sample, the other
sampler / schedule variants of the same workload, and the random-gather
ceiling measured on the device.
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
KERNEL_SOURCES = ["paper_2107_11983_amd/csrc/walk.hip", "paper_2107_11983_amd/csrc/walk_common.hpp",
                  "paper_2107_11983_amd/csrc/trw_device.hpp", "paper_2107_11983_amd/csrc/trw_internal.hpp"]

# Algorithmic bytes: per move the row range
# (two int32 row offsets) 8 B, the sampling entry the move needs and the path
# entry written 4 B; per query the source read, path[0], length and status.
ENTRY_BYTES = {"alias": 12, "naive": 4, "its": None, "orej": None}
PER_QUERY_BYTES = 4 + 4 + 4 + 1


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(tag):
    """HBM bytes per launch (total, read, written) from a committed rocprofv3 counter summary, if current."""
    path = os.path.join(ROOT, "profiles", f"counters_{tag}.md")
    if not os.path.exists(path):
        return None, None
    text = open(path).read()
    kv = dict(re.findall(r"^- (\w+): ([0-9a-fA-F.e+]+)\s*$", text, flags=re.M))
    if kv.get("kernel_source_sha256_16") != kernel_source_hash():
        return None, "stale"
    try:
        return {"total": float(kv["traffic_bytes_per_launch"]), "read": float(kv.get("read_bytes_per_launch", "nan")),
                "write": float(kv.get("write_bytes_per_launch", "nan")),
                "l2_hit_rate": float(kv["l2_hit_rate"]) if "l2_hit_rate" in kv else None}, path
    except KeyError:
        return None, None


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ppr-rmat22")
    ap.add_argument("--sampler", default=None, help="default: the workload's first sampler")
    ap.add_argument("--mode", default="persistent", choices=["persistent", "per_step"])
    ap.add_argument("--wpl", type=int, default=0, help="walkers per lane (0 = library default)")
    ap.add_argument("--blocks-per-cu", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--nq", type=int, default=0, help="override the number of queries (throughput-vs-batch sweeps)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target oracle CPU time")
    ap.add_argument("--serve-requests", type=int, default=10000, help="measured requests (served workload)")
    ap.add_argument("--serve-scale", type=int, default=0, help="override the served graph's scale (tests)")
    ap.add_argument("--serve-slots-per-cu", type=int, default=2048)
    ap.add_argument("--serve-steps", type=int, default=16, help="moves per walker slot per tick")
    ap.add_argument("--serve-pipelined", type=int, default=1, help="0: serial ticks (read each tick before queueing the next)")
    ap.add_argument("--serve-rate", type=float, default=0.0, help="offered requests/s (0: 0.7x the saturated rate)")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for counter collection: a 1 GiB copy (calibration) then the walk only")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this engine runs on one GPU; queries shard across GPUs with no exchange, "
              "since each walk reads only the shared graph, but only the 1-GPU figure is measured. Use --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2107_11983_amd as trw

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    props = torch.cuda.get_device_properties(0)
    log(f"device {props.name} cus={props.multi_processor_count}")

    wl = synth.WORKLOADS[args.workload]
    if wl.algo == "mixed":
        return bench_served(args, wl, np, torch, synth, trw, props)
    sampler = args.sampler or {"metapath": "its+index", "node2vec": "orej+eidx",
                               "deepwalk": "naive+adj"}.get(wl.algo, wl.samplers[0])
    t0 = time.time()
    g = synth.make_graph(wl)
    log(f"graph {wl.name}: n={g.n} m={g.m} dmax={int(g.degrees().max())} ({time.time() - t0:.1f}s)")
    src_np = synth.make_sources(wl, g, nq=args.nq or None)
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
        if args.wpl:
            t["walkers_per_lane"] = args.wpl
        if args.blocks_per_cu:
            t["blocks_per_cu"] = args.blocks_per_cu
        if args.chunk:
            t["queue_chunk"] = args.chunk
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

    mode = trw.MODES[args.mode]
    if args.profile_pass:
        # calibration: a plain device copy of exactly 1 GiB, then the walk
        a = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        r = run(sampler, mode, 1, max(args.steps, 1), tuning_for())
        log(f"profile pass: {r['moves']} moves per launch, {np.mean(r['per_launch_ms']):.3f} ms per launch")
        return

    log(f"main: {wl.algo}/{sampler} {args.mode} warmup={args.warmup} steps={args.steps}")
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
        measured, src = read_traffic(f"{wl.name}_{sampler}_{args.mode}")
        traffic = measured["total"] if measured else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                    "kernel": f"k_walk_persistent<{wl.algo},{sampler}>" if args.mode == "persistent"
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

    # Autotuned launch (the paper's pre-execution tuning): candidates timed on a
    # sample of the batch, then the whole batch timed with the winner.
    autotuned = None
    if not args.no_variants and not args.profile_pass:
        n_tune = min(nq, 1 << 20)
        t0 = time.perf_counter()
        best, best_ms = trw.autotune(G, tables.get(sampler), params(sampler), d_src[:n_tune], mode=mode)
        tune_s = time.perf_counter() - t0
        r = run(sampler, mode, 1, args.steps, best)
        v = r["moves"] * args.steps / r["wall_s"]
        autotuned = {"tuning": best.as_dict(), "sample_queries": n_tune, "tune_s": round(tune_s, 3),
                     "steps_per_s": round(v, 1), "ms_per_batch": round(1000 * r["wall_s"] / args.steps, 4),
                     "vs_default": round(v / value, 4)}
        log(f"autotuned {best.as_dict()}: {v:.4g} steps/s ({v / value:.3f}x default), tuning {tune_s:.2f}s")

    # Other samplers / schedules of the same workload (same queries, same graph).
    variants = {}
    if not args.no_variants:
        for s in variant_samplers:
            for mname in ("persistent", "per_step"):
                if s == sampler and mname == args.mode:
                    continue
                if ((wl.algo in ("ppr", "deepwalk") and s in ("alias", "its", "rej")) or "+" in s) and s not in tables:
                    continue
                r = run(s, trw.MODES[mname], 1, 3)
                v = r["moves"] * 3 / r["wall_s"]
                variants[f"{s}/{mname}"] = {"steps_per_s": round(v, 1), "ms_per_batch": round(1000 * r["wall_s"] / 3, 3),
                                            "moves": r["moves"]}
                log(f"variant {s}/{mname}: {v:.4g} steps/s")
        if wl.algo in ("ppr", "deepwalk") and sampler.startswith("naive") and args.mode == "persistent":
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

    # Random-gather ceiling of the device (dependent and independent chains).
    gather = None
    if not args.no_probe:
        gather = probe_gather(trw, torch, dev, props.multi_processor_count)
        if roofline is not None and gather:
            acc_s = roofline.get("issued_random_reads_per_launch", roofline["random_reads_per_launch"]) / (
                avg_launch_ms * 1e-3)
            roofline["issued_random_reads_per_s"] = round(acc_s, 1)
            roofline["frac_of_dependent_gather_ceiling"] = round(acc_s / gather["dependent_best_reads_per_s"], 4)
            roofline["frac_of_independent_gather_ceiling"] = round(acc_s / gather["independent_best_reads_per_s"], 4)
            # Both halves of the traffic against their measured random ceilings: the issued random
            # reads at the gather rate plus the bytes written (counters) at the 64 B scatter rate.
            if measured and measured["write"] == measured["write"] and gather.get("scatter"):
                t_r = roofline.get("issued_random_reads_per_launch", roofline["random_reads_per_launch"]) / \
                    gather["dependent_best_reads_per_s"]
                t_w = measured["write"] / (gather["scatter"]["64"]["GBps"] * 1e9)
                roofline["random_ceiling_ms"] = round(1e3 * (t_r + t_w), 4)
                roofline["frac_of_random_ceiling"] = round((t_r + t_w) / (avg_launch_ms * 1e-3), 4)

    cpu = cpu_par = None
    if not args.no_cpu_baseline:
        cpu, cpu_par = cpu_baseline(g, wl, sampler, src_np, kw, args.cpu_seconds)

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
        measured, src = read_traffic(f"{wl.name}_{sampler}_{args.mode}")
        traffic = measured["total"] if measured else None
        roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBPS, 5), "traffic": traffic,
                    "kernel": f"k_walk_persistent<{wl.algo},{sampler}>", "alg_bytes_per_launch": alg_bytes,
                    "avg_launch_ms": round(avg_launch_ms, 4), "alg_bytes_per_move": round(per_move, 3),
                    "alg_bytes_from": alg_from}
        if traffic is not None:
            roofline["traffic_frac_of_peak"] = round(traffic / (avg_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
            roofline["l2_hit_rate"] = measured.get("l2_hit_rate")
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
        "config": {"workload": f"{wl.name}: {wl.algo} sampler={sampler} mode={args.mode}; R-MAT 2^{wl.scale} "
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
    print(json.dumps(out), flush=True)


def bench_served(args, wl, np, torch, synth, trw, props):
    """Served mixed workload: Poisson arrivals of requests of 1..4096 queries, each DeepWalk
    (80 moves, ALIAS), PPR (stop 0.2, ALIAS) or Node2Vec (p=2, q=0.5, 80 moves), on a resident
    weighted symmetric R-MAT graph; continuous batching with memory admission and graph-captured
    ticks.  Reports p50/p99 request latency at 0.7x the saturated request rate, and steps/s."""
    import ctypes
    from paper_2107_11983_amd import _abi
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
            adj = tab
    log(f"tables {pre}")
    n_sat, n_warm, n_meas = 2000, 500, args.serve_requests
    n_trials = 4                    # saturation replays: a warm-up, then three timed, each on its own requests
    N = n_trials * n_sat + n_warm + n_meas
    sizes = 1 + synth.uniform_u32(N, 4096, wl.walk_seed ^ 0x5153).astype(np.int64)
    kinds = synth.uniform_u32(N, 3, wl.walk_seed ^ 0xA160)
    offs = np.concatenate([[0], np.cumsum(sizes)])
    d_src = torch.from_numpy(synth.sources(int(offs[-1]), g.n, wl.src_seed)).cuda()
    algo_p = [trw.make_params("deepwalk", "alias", 80, wl.walk_seed),
              trw.make_params("ppr", "alias", 256, wl.walk_seed, stop_q32=trw.stop_threshold(0.2)),
              trw.make_params("node2vec", "orej", 80, wl.walk_seed, n2v_thr_q16=trw.n2v_thresholds(2.0, 0.5))]
    strides = [88, 264, 88]
    path_off = np.concatenate([[0], np.cumsum(sizes * np.array(strides)[kinds])])
    d_paths = torch.empty(int(path_off[-1]), dtype=torch.int32, device="cuda")
    d_len = torch.empty(int(offs[-1]), dtype=torch.int32, device="cuda")
    d_st = torch.empty(int(offs[-1]), dtype=torch.uint8, device="cuda")
    reqs = (_abi.trw_request * N)()
    for i in range(N):
        r = reqs[i]
        r.params = algo_p[kinds[i]]
        r.nq = int(sizes[i])
        r.sources = ctypes.c_void_p(d_src.data_ptr() + 4 * int(offs[i]))
        r.qid_base = i << 32
        r.paths = ctypes.c_void_p(d_paths.data_ptr() + 4 * int(path_off[i]))
        r.path_stride = strides[kinds[i]]
        r.lengths = ctypes.c_void_p(d_len.data_ptr() + 4 * int(offs[i]))
        r.status = ctypes.c_void_p(d_st.data_ptr() + int(offs[i]))
    torch.cuda.synchronize()
    slots = props.multi_processor_count * args.serve_slots_per_cu
    srv = trw.Server(G, alias, adj, pool_bytes=8 << 30, max_slots=slots, max_requests=1024,
                     steps_per_tick=args.serve_steps, pipelined=bool(args.serve_pipelined))

    def replay(lo, hi, arrivals):
        comp = (_abi.trw_completion * (hi - lo))()
        arr = (ctypes.c_uint64 * (hi - lo))(*[int(x) for x in arrivals])
        m0 = srv.stats()["moves"]
        t = time.perf_counter()
        rc = _abi.trw_probe_serve_replay(srv.handle, hi - lo, ctypes.byref(reqs, ctypes.sizeof(_abi.trw_request) * lo),
                                         arr, comp, 600_000)
        wall = time.perf_counter() - t
        assert rc == 0, f"replay failed: {rc} {_abi.trw_last_error()}"
        assert all(comp[i].status == 0 for i in range(hi - lo))
        return comp, wall, srv.stats()["moves"] - m0

    # saturation: everything arrives at once; a warm-up replay, then the
    # median of three (one 20 ms replay varies by tens of percent), each on
    # requests of its own so that no replay finds the previous one's rows cached
    trials = []
    for rep in range(n_trials):
        comp, wall, moves = replay(rep * n_sat, (rep + 1) * n_sat, np.zeros(n_sat))
        if rep:
            trials.append((wall, moves))
    wall, moves = sorted(trials)[1]
    sat_rps = n_sat / wall
    sat_steps = moves / wall
    st0 = srv.stats()
    log(f"saturated: {n_sat} requests in {wall:.3f}s (median of {[round(n_sat / w) for w, _ in trials]} req/s) = "
        f"{sat_rps:.0f} req/s, {sat_steps:.4g} steps/s; {st0['ticks']} ticks, device {st0['tick_device_ns'] / 1e6:.1f} ms")
    # offered load 0.7x saturation (or a fixed rate), Poisson arrivals (exponential gaps from seeded uniforms)
    rate = args.serve_rate or 0.7 * sat_rps
    u = synth.uniform_f64(n_warm + n_meas, wl.walk_seed ^ 0x9015)
    arrivals = np.cumsum(-np.log(u) / rate) * 1e9
    comp, wall, moves = replay(n_trials * n_sat, N, arrivals - arrivals[0])
    lat = np.array([(comp[i].t_done_ns - comp[i].t_submit_ns) / 1e6 for i in range(n_warm, n_warm + n_meas)])
    queue = np.array([(comp[i].t_admit_ns - comp[i].t_submit_ns) / 1e6 for i in range(n_warm, n_warm + n_meas)])
    span = (comp[n_warm + n_meas - 1].t_done_ns - comp[n_warm].t_submit_ns) / 1e9
    st = srv.stats()
    srv.close()
    out = {
        "metric": "walk steps/sec + % HBM roofline (1 GPU); p50/p99 query latency served",
        "value": round(moves / wall, 1), "unit": "steps/s", "n_gpus": 1, "steps": n_meas, "warmup": n_warm,
        "ms_per_step": round(1000 * wall / (n_warm + n_meas), 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": f"{wl.name}: served mix of DeepWalk-80 ALIAS / PPR-0.2 ALIAS / Node2Vec p=2 q=0.5 "
                               f"len 80, requests of U{{1..4096}} queries, Poisson arrivals at "
                               f"{'%.0f req/s' % args.serve_rate if args.serve_rate else '0.7x saturation'}; "
                               f"R-MAT 2^{int(np.log2(g.n))} symmetric avg deg {wl.avg_degree}, uint32 weights 1..255",
                   "n": g.n, "m": g.m, "parallelism": "1 GPU"},
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3), "p99": round(float(np.percentile(lat, 99)), 3),
                       "mean": round(float(lat.mean()), 3), "queue_p50": round(float(np.percentile(queue, 50)), 3),
                       "queue_p99": round(float(np.percentile(queue, 99)), 3)},
        "offered_req_per_s": round(rate, 1), "achieved_req_per_s": round(n_meas / span, 1),
        "saturated": {"req_per_s": round(sat_rps, 1), "steps_per_s": round(sat_steps, 1),
                      "trials_req_per_s": [round(n_sat / w, 1) for w, _ in trials]},
        "server": {"ticks": st["ticks"], "steps_per_tick": args.serve_steps, "slots": slots,
                   "pipelined": bool(args.serve_pipelined),
                   "max_requests": 1024, "pool_bytes": st["pool_bytes"],
                   "tick_device_ms_mean": round(st["tick_device_ns"] / max(st["ticks"], 1) / 1e6, 4)},
        "preprocess_ms": pre,
    }
    print(json.dumps(out), flush=True)


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
    res["dependent_best_GBps_at_64B"] = round(best[1] * 64 / 1e9, 1)
    res["independent_best_GBps_at_64B"] = round(best[0] * 64 / 1e9, 1)
    log(f"gather ceiling: dependent {best[1]:.4g} reads/s, independent {best[0]:.4g} reads/s")
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
    single = {"value": round(moves / dt, 1), "unit": "steps/s", "cores": 1, "kind": "oracle",
              "sample": f"first {nsamp} of {len(src_np)} queries of the same batch ({moves} moves, {dt:.1f} s, "
                        f"single thread, tables prebuilt)", "oracle_counters": counters}
    # The same sample sharded by query range over the host's cores (the
    # oracle unchanged; ctypes releases the interpreter lock during each call).
    import concurrent.futures
    workers = max(1, min(16, os.cpu_count() or 1))
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
                          f"({pdt:.1f} s)"}
    return single, parallel


if __name__ == "__main__":
    main()

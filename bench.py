#!/usr/bin/env python3
"""Benchmark of the contig-generation path on one MI355X.

One step = one pass of the whole path (branch removal, connected components,
LPT partitioning, induced subgraphs, local assembly) over one batch of
synthetic string graphs already resident in HBM.  The default workload is the
batched configuration: 512 independent graphs (genomes log-uniform in
0.2-20 Mbp, 10-40x coverage, reads lognormal with mean 10 kbp and sd 3 kbp,
0.5-3% extra branch edges, P = 64 bins per graph).

Printed on the last stdout line, as JSON: throughput in contig bases/s, the
string-graph edges/s of the mask + components phase, the roofline of the
dominant kernel (HIP events, algorithmic bytes) and the oracle's CPU
throughput on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch|plain50|large1g]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "string-graph edges/s + contig bases/s, batched vs plain, % of HBM peak"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# Algorithmic bytes per kernel (each array counted once; gathers, re-reads and
# atomics traffic are not counted).  `s` holds the workload's sizes for the
# graphs one launch processes.
# ---------------------------------------------------------------------------

def algo_bytes(kernel, s):
    N, m, m_nb, n_e, m_e, nc, Cb, W = (s["N"], s["m"], s["m_nb"], s["n_e"], s["m_e"], s["n_comp"],
                                       s["contig_bases"], s["words"])
    table = {
        # row_ptr (N+1), the columns of rows of degree <= 2, flags written
        "k_mask": 4 * (N + 1) + 4 * m_nb + N,
        "k_cc_init": 4 * N,
        # flags + row_ptr + kept columns read; label updates not counted
        "k_cc_hook": N + 4 * N + 4 * m_nb,
        "k_cc_compress": 4 * N + 4 * N,
        # the batched mask + components kernel: row_ptr, the columns of rows of
        # degree <= 2, flags, labels and label_comp written, the component
        # table (label, size, kind, member start) and the grouped members
        "k_mask_cc": 4 * (N + 1) + 4 * m_nb + N + 4 * N + 4 * N + 13 * nc + 4 * n_e,
        "k_part_zero": 4 * N,
        "k_part_count": N + 4 * N,
        "k_part_compact": N + 4 * N + 4 * N + 9 * nc,
        "k_part_lpt": 4 * nc + 16 * nc,
        "k_ind_zero": 4 * nc,
        "k_ind_fill": 4 * N + 4 * N + 8 * n_e,
        "k_ind_local": 8 * n_e + 4 * n_e,
        "k_ind_rows": 4 * n_e + n_e + 4 * (n_e + 1) + 8 * m_e + 4 * n_e,
        "k_ind_rows_wide": 4 * n_e + n_e + 4 * (n_e + 1) + 8 * m_e + 4 * n_e,
        # perm, local rows, entries (columns + ids, strands + overlaps), read
        # lengths and store offsets; layout (id, strand) and pieces (length,
        # store anchor, offset) written
        "k_asm_walk": 4 * n_e + 8 * n_e + 8 * m_e + 9 * m_e + 12 * n_e + 5 * n_e + 20 * n_e,
        "k_asm_offsets": 16 * nc,
        # packed source bases read + contig words written + per-piece
        # descriptors (contig, offset, length, store anchor) and per-contig
        # records (length, base offset)
        "k_asm_copy": Cb // 4 + 4 * W + 24 * n_e + 16 * nc,
    }
    return table.get(kernel)


# least CPU time the oracle baselines are timed over (whole passes over the
# workload's graphs), so that the figure is not a sub-second measurement
MIN_CPU_SECONDS = 10.0


def csrc_digest():
    """sha256 over the kernel sources, in the order the byte-counter profile uses."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2207_04350_amd", "csrc", "*"))):
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


# counter profiles of the single-graph workloads' plain form
PLAIN_PROFILES = {"large1g": "plain_1gbp_hbm_bytes.md"}


def profiled_traffic(kernel, profile="batched_512graphs_hbm_bytes.md"):
    """HBM bytes per launch of a kernel from a committed counter profile
    (scaled FETCH_SIZE + WRITE_SIZE), or None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", profile)
    if not os.path.exists(path):
        return None
    digest, mb = None, None
    with open(path) as f:
        for line in f:
            if line.startswith("csrc sha256:"):
                digest = line.split(":", 1)[1].strip()
            cells = [c.strip() for c in line.split("|")]
            if len(cells) >= 5 and cells[1].strip("`").startswith("cg::%s(" % kernel):
                mb = float(cells[4])
    if digest != csrc_digest() or mb is None:
        return None
    return mb * 1e6


def workload_graphs(name):
    import synth
    if name == "batch":
        return synth.batch_graphs(512), "batched: 512 independent string graphs (genome 0.2-20 Mbp " \
            "log-uniform, 10-40x, reads LN(10k,3k), 0.5-3% branch edges, P=64 per graph)"
    if name == "plain50":
        return [synth.config_graph(2)], "plain: one string graph, 50 Mbp genome + 200x8 kbp " \
            "repeats, 30x, reads LN(12k,4k), 2% branch edges, P=64"
    if name == "large1g":
        return [synth.config_graph(3)], "plain: one string graph, 1 Gbp genome with 5% repeats, " \
            "20x, reads LN(15k,5k), 1% branch edges, P=1024"
    raise SystemExit("unknown workload %s" % name)


def host_info():
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "usable_cpus": len(os.sched_getaffinity(0)),
            "cpu_model": model}


def _pool_worker(src, idx, Ps, barrier, q):
    import oracle
    import synth
    # this worker's graphs, regenerated from their seeds: graphs idx of the
    # batched workload, or requests idx of the serving pool of src[1]
    if src[0] == "batch":
        gs = synth.batch_graphs(512, only=idx)
    else:
        recipes = synth.request_params(src[1])
        gs = [synth.simulate(**recipes[i]) for i in idx]
    barrier.wait()
    t0 = time.perf_counter()
    bases, busy = 0, 0.0
    for g, P in zip(gs, Ps):
        tm = {}
        bases += int(oracle.run(g, P=P, min_reads=2, timings=tm)["contigs"]["len"].sum())
        busy += tm["total"]
    q.put((bases, time.perf_counter() - t0, len(gs), busy))


def cpu_pool_baseline(graphs, Ps, workers, src=("batch", 512)):
    """The single-threaded oracle in `workers` processes, one graph at a time
    per process (graph-level parallelism only); graphs go to workers by LPT on
    their read counts.  Wall time runs from a barrier all workers reach after
    building their inputs to the last worker's end.  src names where the
    workers regenerate the graphs from: ("batch", 512) for the batched
    workload (graph k is the generator's graph of its name), ("request", n)
    for the serving pool of n requests (graph k is request k)."""
    import multiprocessing as mp
    mpc = mp.get_context("spawn")
    load = [0] * workers
    part = [[] for _ in range(workers)]
    # graph k of the list is graph ids[k] of the batched workload's generator
    ids = [int(g.meta["name"].rsplit("-", 1)[1]) for g in graphs] if src[0] == "batch" \
        else list(range(len(graphs)))
    for i in sorted(range(len(graphs)), key=lambda i: (-graphs[i].n, i)):
        w = min(range(workers), key=lambda w: (load[w], w))
        part[w].append(i)
        load[w] += graphs[i].n
    barrier, q = mpc.Barrier(workers + 1), mpc.Queue()
    procs = [mpc.Process(target=_pool_worker,
                         args=(src, [ids[i] for i in part[w]], [Ps[i] for i in part[w]], barrier,
                               q))
             for w in range(workers) if part[w]]
    barrier = barrier if len(procs) == workers else None
    if barrier is None:
        raise RuntimeError("fewer graphs than workers")
    for pr in procs:
        pr.start()
    barrier.wait(timeout=600)
    t0 = time.perf_counter()
    res = [q.get(timeout=600) for _ in procs]
    wall = time.perf_counter() - t0
    for pr in procs:
        pr.join()
    bases = sum(r[0] for r in res)
    busiest = max(r[3] for r in res)
    # timed like the single-threaded baseline: the C oracle's own clock, here
    # that of the busiest worker; the wall time adds the Python marshalling
    return {"value": bases / busiest, "unit": "contig bases/s", "cores": workers,
            "kind": "oracle",
            "sample": "all %d graphs (%d contig bases), %d processes of the single-threaded C "
                      "oracle, one graph at a time each" % (len(graphs), bases, workers),
            "seconds": busiest, "wall_s": wall,
            "timing": "C oracle phase clocks of the busiest worker (wall_s: barrier to last "
                      "result, Python marshalling included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="batch", choices=["batch", "plain50", "large1g", "serve", "reduce"])
    ap.add_argument("--requests", type=int, default=1000, help="serve: measured requests")
    ap.add_argument("--max-wave", type=int, default=64, help="serve: requests per wave at most")
    ap.add_argument("--lane-bytes", type=int, default=2 << 30,
                    help="serve: batch memory of each of the two lanes")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="bound on the oracle's CPU baseline sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-workers", type=int,
                    default=min(16, len(os.sched_getaffinity(0))),
                    help="processes of the oracle pool baseline (batched and serving workloads)")
    ap.add_argument("--shape", default="",
                    help="vertex_tile,copy_block,persist_blocks of the batched form (skips tuning)")
    ap.add_argument("--skip-plain", action="store_true",
                    help="profile runs: leave out the plain per-graph form")
    ap.add_argument("--reps", type=int, default=20,
                    help="repetitions behind the median per-kernel timings (warm and cold)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device a few times (the reference kernel "
                         "that scales HBM byte counters), then exit")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        src = torch.ones(args.copy_calibration << 18, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copied %d MiB 3 times" % args.copy_calibration)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the path runs on one GPU's share of "
              "the graphs and has no multi-GPU mode (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2207_04350_amd import cg

    if args.workload == "serve":
        return serve_bench(args)
    if args.workload == "reduce":
        return reduce_bench(args)

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cg.lib()

    t0 = time.time()
    graphs, desc = workload_graphs(args.workload)
    log("generated %d graphs in %.1fs" % (len(graphs), time.time() - t0))
    Ps = [g.meta["P"] for g in graphs]
    t0 = time.time()
    dgs = [cg.DeviceGraph(g, dev) for g in graphs]
    outs = [cg.Outputs(g.n, P, g.seq_words, dev) for g, P in zip(graphs, Ps)]
    big = max(range(len(graphs)), key=lambda i: cg.footprint(graphs[i].n, graphs[i].m, Ps[i]))
    ctx = cg.Context.for_graph(graphs[big].n, graphs[big].m, Ps[big])
    torch.cuda.synchronize()
    log("resident in HBM in %.1fs" % (time.time() - t0))
    stream = torch.cuda.current_stream()

    jobs = [(dg, out, P, 2) for dg, out, P in zip(dgs, outs, Ps)]

    def plain_step():
        for dg, out, P in zip(dgs, outs, Ps):
            cg.run_path(ctx, dg, out, P, 2, stream)

    def timed(step, stream_, steps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream_)
        for _ in range(steps):
            step()
        e1.record(stream_)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps, e0.elapsed_time(e1) / steps

    # a buffer larger than the 256 MB Infinity Cache: writing it before a rep
    # leaves none of the path's data in cache ("cold")
    flush = torch.empty(1 << 28, dtype=torch.int32, device=dev)

    def timed_cold(step, stream_, steps):
        """K steps, each after a 1 GiB write on the same stream (the cache then
        holds none of the path's data): the mean time of a step between HIP
        events recorded around it on the stream."""
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        tot = 0.0
        with torch.cuda.stream(stream_):
            for k in range(steps):
                flush.fill_(k)
                e0.record(stream_)
                step()
                e1.record(stream_)
                stream_.synchronize()
                tot += e0.elapsed_time(e1)
        torch.cuda.synchronize()
        return tot / steps

    def kernel_reps(step, stream_, reps, cold):
        """Median over reps of each kernel's per-step time, and of the step's
        time between events; cold reps flush the cache first."""
        per, whole = [], []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for r in range(reps):
            if cold:
                flush.fill_(r)
            ctx.profile(64)
            e0.record(stream_)
            step()
            e1.record(stream_)
            prof = ctx.profile_read()
            ctx.profile(0)
            torch.cuda.synchronize()
            whole.append(e0.elapsed_time(e1))
            per.append({k: v[1] for k, v in prof.items() if k[0] != "_"})
        keys = sorted(set().union(*per))
        return ({k: float(np.median([p.get(k, 0.0) for p in per])) for k in keys},
                float(np.median(whole)))

    def kernel_profile(step, steps, launches_per_step):
        ctx.profile(launches_per_step * steps + 64)
        for _ in range(steps):
            step()
        prof = ctx.profile_read()
        ctx.profile(0)
        return {k: (c / steps, ms / steps) for k, (c, ms) in prof.items() if k[0] != "_"}

    # ---- plain per-graph launches -----------------------------------------
    if not args.skip_plain:
        for _ in range(args.warmup):
            plain_step()
        plain_wall, plain_gpu = timed(plain_step, stream, args.steps)
        plain_cold = timed_cold(plain_step, stream, args.steps)
        log("plain: %.3f ms/step wall, %.3f ms/step between events, %.3f ms/step cold"
            % (plain_wall, plain_gpu, plain_cold))
        plain_kern = kernel_profile(plain_step, args.steps, 16 * len(graphs))
    else:
        plain_wall = plain_gpu = plain_cold = float("nan")
        plain_kern = {}

    # ---- batched: tuned launch shapes, one HIP graph per step ---------------
    from paper_2207_04350_amd import autotune
    side = torch.cuda.Stream()
    t0 = time.time()
    if args.shape:
        shape, table = tuple(int(x) for x in args.shape.split(",")), {}
    else:
        shape, table = autotune.tune(ctx, jobs, side, use_cache=False, log=log)
    log("tuned %s in %.1fs" % (shape, time.time() - t0))
    batch = cg.Batch(ctx, jobs, *shape)
    with torch.cuda.stream(side):
        batch.capture(side)
    with torch.cuda.stream(side):
        for _ in range(args.warmup):
            batch.launch(side)
        b_wall, b_gpu = timed(lambda: batch.launch(side), side, args.steps)
    log("batched: %.3f ms/step wall, %.3f ms/step between events" % (b_wall, b_gpu))

    b_cold = timed_cold(lambda: batch.launch(side), side, args.steps)
    log("batched, HIP graph after a cache flush: %.3f ms/step (mean of %d)" % (b_cold, args.steps))
    with torch.cuda.stream(side):
        batch_kern = kernel_profile(lambda: batch.run(side), args.steps, 16)
        # medians of per-kernel times, warm and cold (the primary mask+CC
        # number is cold: the cache would otherwise hold its whole working set)
        for _ in range(3):
            batch.run(side)
        warm_k, warm_step = kernel_reps(lambda: batch.run(side), side, args.reps, False)
        cold_k, cold_step = kernel_reps(lambda: batch.run(side), side, args.reps, True)
    log("batched, median of %d: warm %.3f ms/step, cold %.3f ms/step (eager launches with "
        "per-kernel events)" % (args.reps, warm_step, cold_step))
    assert ctx.status(side) == 0, "device status raised"

    # ---- workload sizes (from one step's device-side counts) ---------------
    st = dict(N=0, m=0, m_nb=0, n_e=0, m_e=0, n_comp=0, contig_bases=0, words=0)
    for g, out in zip(graphs, outs):
        deg = np.diff(g.row_ptr)
        st["N"] += g.n
        st["m"] += g.m
        st["m_nb"] += int(deg[deg <= 2].sum())
        sz = out.sizes.cpu().numpy()
        st["n_e"] += int(sz[0])
        st["m_e"] += int(sz[1])
        nc = int(out.n_comp.item())
        st["n_comp"] += nc
        st["contig_bases"] += int(out.c_len[:nc].sum().item())
        st["words"] += int(out.total_words.item())

    def phases(kern):
        pick = lambda pred: sum(v[1] for k, v in kern.items() if pred(k))
        return {
            # the batched form: degrees, bitmaps and lists over the whole chip
            # (kb_mask_tiles), then kept entries, labels and the component
            # table per graph (kb_mask_cc, counted here as components)
            "mask": pick(lambda k: k in ("k_mask", "kb_mask_tiles")),
            "components": pick(lambda k: k.startswith("k_cc") or k == "kb_mask_cc"),
            "partition": pick(lambda k: k.startswith("k_part") or k.startswith("kb_weight")
                              or k in ("kb_lpt", "kb_tables", "kb_wq_place")),
            "induce": pick(lambda k: k.startswith("k_ind")),
            # the batched form induces and walks components of up to 1024
            # reads in one pass (and induces the larger ones in it)
            "induce_walk": pick(lambda k: k.startswith("kb_induce_walk")),
            "assemble": pick(lambda k: k.startswith("k_asm") or k.startswith("kb_walk")
                             or k in ("kb_offsets", "kb_copy")),
        }

    def medians(km):
        return phases({k: (1, v) for k, v in km.items()})

    for name, kern in (("plain", plain_kern), ("batched", batch_kern)):
        for k, (c, ms) in sorted(kern.items(), key=lambda kv: -kv[1][1]):
            log("  %-8s %-22s %6d launches/step %9.3f ms/step %9.2f us/launch"
                % (name, k, c, ms, 1e3 * ms / c))

    b_ph = phases(batch_kern)
    warm_ph, cold_ph = medians(warm_k), medians(cold_k)
    maskcc_ms = b_ph["mask"] + b_ph["components"]
    # fused minimum of mask + components: row_ptr, the columns of degree <= 2
    # rows, flags written, labels written (each array once)
    maskcc_bytes = 4 * (st["N"] + 1) + 4 * st["m_nb"] + st["N"] + 4 * st["N"]

    mc = [profiled_traffic(k) for k in ("kb_mask_tiles", "kb_mask_cc")]
    maskcc_traffic = sum(mc) if all(t is not None for t in mc) and args.workload == "batch" else None

    def maskcc(ph):
        ms = ph["mask"] + ph["components"]
        return {"ms": ms, "edges_per_s": st["m"] / (ms * 1e-3),
                "hbm_frac": maskcc_bytes / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}
    kname = lambda k: k.replace("kb_", "k_").replace("<T>", "")
    # a single graph: the faster of the two forms is the reported one (the
    # batched form is built for many graphs; one large graph is the plain
    # path's case)
    use_plain = len(graphs) == 1 and plain_cold == plain_cold and plain_cold < b_cold
    # the step is cold (the cache flushed before each step), the primary
    # figure; the warm one (back-to-back steps) is reported beside it
    step_ms = plain_cold if use_plain else b_cold
    warm_ms = plain_wall if use_plain else b_wall
    form = ("plain: the five cg_* calls on one stream" if use_plain else
            "batched: one HIP graph of %d launches for all graphs"
            % int(round(sum(v[0] for v in batch_kern.values()))))
    rkern = plain_kern if use_plain else batch_kern
    dom = max(rkern, key=lambda k: rkern[k][1])
    dom_launches, dom_ms = rkern[dom]
    dom_avg_us = 1e3 * dom_ms / dom_launches
    dom_map = {"kb_copy": ["k_asm_copy"], "kb_walk": ["k_asm_walk"], "kb_lpt": ["k_part_lpt"],
               "kb_induce_walk": ["k_ind_local", "k_ind_rows", "k_asm_walk"],
               "kb_induce_walk_small": ["k_ind_local", "k_ind_rows", "k_asm_walk"],
               "kb_offsets": ["k_asm_offsets"]}
    dom_bytes = sum(algo_bytes(k, st) or 0 for k in dom_map.get(dom, [kname(dom)]))
    dom_bytes_per_launch = (dom_bytes or 0) / dom_launches
    achieved = dom_bytes_per_launch / (dom_avg_us * 1e-6) / 1e9

    result = {
        "metric": METRIC,
        "value": st["contig_bases"] / (step_ms * 1e-3),
        "unit": "contig bases/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_ms,
        "cache": "cold: a 1 GiB write before each timed step; warm_ms_per_step: "
                 "back-to-back steps",
        "warm_ms_per_step": warm_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded simulated genomes and reads; exact reduced string graphs)",
        "config": {"workload": desc,
                   "form": form,
                   "graphs": len(graphs), "reads": st["N"], "directed_entries": st["m"],
                   "contig_reads": st["n_e"], "contigs": st["n_comp"],
                   "contig_bases": st["contig_bases"],
                   "packed_read_bytes": int(sum(g.seq_words for g in graphs) * 4),
                   "launch_shape": {"vertex_tile": shape[0], "copy_block": shape[1],
                                    "persist_blocks": shape[2]}},
        "batched": {"ms_per_step": b_wall, "gpu_ms_per_step": b_gpu, "cold_ms_per_step": b_cold,
                    "contig_bases_per_s": st["contig_bases"] / (b_wall * 1e-3),
                    "phase_kernel_ms": b_ph,
                    "median_of": args.reps,
                    "warm": {"ms_per_step": warm_step, "phase_kernel_ms": warm_ph,
                             "kernel_ms": warm_k,
                             "contig_bases_per_s_assemble":
                                 st["contig_bases"] / (warm_ph["assemble"] * 1e-3)},
                    "cold": {"ms_per_step": cold_step, "phase_kernel_ms": cold_ph,
                             "kernel_ms": cold_k,
                             "contig_bases_per_s": st["contig_bases"] / (cold_step * 1e-3),
                             "contig_bases_per_s_assemble":
                                 st["contig_bases"] / (cold_ph["assemble"] * 1e-3),
                             "flush": "1 GiB written before each rep"}},
        "plain": {"ms_per_step": plain_wall, "gpu_ms_per_step": plain_gpu,
                  "cold_ms_per_step": plain_cold,
                  "contig_bases_per_s": st["contig_bases"] / (plain_wall * 1e-3),
                  "phase_kernel_ms": phases(plain_kern)},
        "batched_vs_plain": plain_cold / b_cold,
        "edges_per_s_mask_cc": st["m"] / (maskcc_ms * 1e-3) if maskcc_ms else None,
        "mask_cc": {"ms_per_step": maskcc_ms, "algorithmic_bytes": maskcc_bytes,
                    "hbm_frac": maskcc_bytes / (maskcc_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
                    if maskcc_ms else None,
                    "cold_median": maskcc(cold_ph), "warm_median": maskcc(warm_ph),
                    "kernels": "kb_mask_tiles (degrees, bitmaps, every read's default flags, "
                               "label and label_comp, and the reads of degree 1-2 with their "
                               "columns, over the whole chip) + kb_mask_cc (one workgroup per "
                               "graph: kept entries, union-find in LDS, the component table and "
                               "its members, what the reads of degree 1-2 change)",
                    # what the phase's kernels move in all (the calibrated
                    # counters of the committed profile): random lines and the
                    # arrays the later steps need, far above the fused minimum
                    "counter_traffic_bytes": maskcc_traffic,
                    "counter_traffic_frac": maskcc_traffic / (maskcc_ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
                    if maskcc_traffic and maskcc_ms else None},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (profiled_traffic(kname(dom).replace("k_", "kb_", 1))
                                 if args.workload == "batch" and not use_plain else
                                 profiled_traffic(kname(dom), PLAIN_PROFILES[args.workload])
                                 if use_plain and args.workload in PLAIN_PROFILES else None),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0, "
                                     "profiles/%s)" % (PLAIN_PROFILES.get(args.workload)
                                                       if use_plain else
                                                       "batched_512graphs_hbm_bytes.md"),
                     "avg_launch_us": dom_avg_us, "bytes_per_launch": dom_bytes_per_launch,
                     "timing": "HIP events around each launch on its stream, %d eager steps"
                               % args.steps},
        "autotune": table,
    }

    # ---- CPU oracle on a bounded sample, with parity of the same graphs ----
    if not args.no_cpu:
        import oracle
        from tests.parity import mismatches
        # whole passes over the graphs (parity checked on the first) until
        # the oracle has run for at least MIN_CPU_SECONDS, at most
        # --cpu-seconds
        spent, bases, done, ok, passes = 0.0, 0, 0, 0, 0
        floor = min(MIN_CPU_SECONDS, args.cpu_seconds)
        while spent < floor:
            for i, g in enumerate(graphs):
                tm = {}
                want = oracle.run(g, P=Ps[i], min_reads=2, timings=tm)
                spent += tm["total"]
                bases += int(want["contigs"]["len"].sum())
                if passes == 0:
                    done += 1
                    got = cg.to_host(outs[i], g.n)
                    ok += int(mismatches(got, want) == [])
                if spent >= args.cpu_seconds:
                    break
            passes += 1
            if spent >= args.cpu_seconds:
                break
        result["cpu_baseline"] = {
            "value": bases / spent, "unit": "contig bases/s", "cores": 1, "kind": "oracle",
            "sample": "%d pass(es) over graphs 0..%d of the %d (%d contig bases in all), "
                      "single-threaded C oracle, whole path" % (passes, done - 1, len(graphs),
                                                                bases),
            "seconds": spent}
        result["parity_sample"] = {"graphs": done, "identical": ok}
        log("oracle: %d graphs in %.1fs, parity %d/%d" % (done, spent, ok, done))
        result["host"] = host_info()
        if args.workload == "batch" and args.cpu_workers > 1:
            pool = cpu_pool_baseline(graphs, Ps, args.cpu_workers)
            result["cpu_baseline_pool"] = pool
            log("oracle pool: %d processes, %.2fs wall" % (args.cpu_workers, pool["seconds"]))
    print(json.dumps(result), flush=True)


def reduce_bench(args):
    """The step before the path: contained-read pruning and transitive
    reduction (cg_reduce) of the overlap graph of the 50 Mbp workload's reads
    (every pair overlapping by >= 1000 bases, contained reads included)."""
    import numpy as np
    import torch

    import synth
    from paper_2207_04350_amd import cg

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    cg.lib()
    t0 = time.time()
    g = synth.config_graph(2)
    r = synth.overlap_graph(g)
    log("overlap graph: n=%d, %d entries (string graph: %d) in %.1fs"
        % (r.n, r.m, g.m, time.time() - t0))
    ctx = cg.Context.for_graph(r.n, r.m, 1)
    dg = cg.DeviceGraph(r, dev)
    out = cg.Reduced(r.n, r.m, dev)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        cg.reduce(ctx, dg, out, 0, stream)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        cg.reduce(ctx, dg, out, 0, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    ms = e0.elapsed_time(e1) / args.steps
    assert ctx.status(stream) == 0, "device status raised"
    ctx.profile(8 * args.reps + 8)
    for _ in range(args.reps):
        cg.reduce(ctx, dg, out, 0, stream)
    prof = {k: v for k, v in ctx.profile_read().items() if k[0] != "_"}
    ctx.profile(0)
    m_s = int(out.d_m.item())
    identical = m_s == g.m and np.array_equal(out.col[:m_s].cpu().numpy(), g.col)
    for k, (c, kms) in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        log("  reduce %-16s %4d launches %9.3f ms/step" % (k, c, kms / args.reps))
    n, m = r.n, r.m
    # each array once: R's row_ptr, col, ovl, strand and read lengths read;
    # contained, kept and the string graph written
    algo = 4 * (n + 1) + 9 * m + 4 * n + n + m + 4 * (n + 1) + 9 * m_s
    dom = max(prof, key=lambda k: prof[k][1])
    dom_us = 1e3 * prof[dom][1] / prof[dom][0]
    # the dominant kernel's own share: R read once, marks written
    dom_bytes = {"k_red_trans": 4 * (n + 1) + 9 * m + 4 * n + n + m}.get(dom, algo)
    result = {
        "metric": "overlap-graph entries/s (contained-read pruning + transitive reduction)",
        "value": m / (wall * 1e-3),
        "unit": "entries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall,
        "gpu_ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded simulated genome and reads; exact overlaps >= 1000 bases)",
        "config": {"workload": "overlap graph of the 50 Mbp + 200x8 kbp repeats, 30x, "
                               "LN(12k,4k) reads (125,000 reads)",
                   "reads": n, "entries": m, "string_graph_entries": m_s,
                   "equals_generator_string_graph": bool(identical)},
        "kernels_ms": {k: v[1] / args.reps for k, v in prof.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": dom_bytes / (dom_us * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": dom_bytes / (dom_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(dom, "reduce_50mbp_hbm_bytes.md"),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE "
                                     "x1.0, profiles/reduce_50mbp_hbm_bytes.md)",
                     "avg_launch_us": dom_us, "bytes_per_launch": dom_bytes,
                     "note": "k_red_trans re-reads each neighbour's row once per row that "
                             "holds it (sum of squared degrees), bound by those lookups"},
    }
    if not args.no_cpu:
        import oracle
        passes = 0
        t0 = time.perf_counter()
        while True:
            oc, ok, os_ = oracle.reduce(r)
            passes += 1
            sec = time.perf_counter() - t0
            if sec >= min(MIN_CPU_SECONDS, args.cpu_seconds):
                break
        result["cpu_baseline"] = {
            "value": passes * m / sec, "unit": "entries/s", "cores": 1, "kind": "oracle",
            "sample": "%d passes over the whole overlap graph, single-threaded C oracle" % passes,
            "seconds": sec}
        result["parity"] = {
            "kept_identical": bool(np.array_equal(out.kept[:m].cpu().numpy(), ok)),
            "contained_identical": bool(np.array_equal(out.contained[:n].cpu().numpy(), oc))}
    ctx.close()
    print(json.dumps(result), flush=True)


def serve_bench(args):
    """Continuous-batching serving of contig-generation requests: a pool of
    synthetic request graphs (genome 1-100 Mbp log-uniform, 15-30x, reads
    LN(12k, 4k), 1-2% branch edges, P = 64) and a seeded Poisson stream
    sampling the pool.  Admitted requests are served in waves, each wave one
    batched launch sequence (cg_batch_plan + cg_batch_run) on one of two
    lanes.  The arrival rate is searched for a device-busy fraction of about
    0.8, device busy measured from GPU events around each wave's launches;
    p50 / p99 latency runs from arrival to the result in host memory.
    Measured with the pool resident in HBM (the reported value) and with
    every request uploading its graph (with_upload).  Every measured
    request's contigs are compared with the oracle's for its graph."""
    import numpy as np
    import torch

    import oracle
    import synth
    from paper_2207_04350_amd import cg, serve

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cg.lib()
    t0 = time.time()
    n_pool = 48
    pool = [serve.HostGraph(synth.simulate(**p)) for p in synth.request_params(n_pool)]
    log("request pool: %d graphs (%.1f M reads, %.1f GB packed reads) in %.1fs" % (
        n_pool, sum(h.n for h in pool) / 1e6, sum(h.seq_words for h in pool) * 4 / 1e9,
        time.time() - t0))
    # the oracle's contigs of every pool graph (parity), timed (cpu_baseline)
    wants, spent = [], 0.0
    for h in pool:
        tm = {}
        wants.append(oracle.run(h.graph, P=64, min_reads=2, timings=tm)["contigs"])
        spent += tm["total"]
    log("oracle over the pool: %.1fs" % spent)
    fields = ("label", "bin", "start", "n_reads", "len", "base_off", "cflags", "layout_off",
              "layout_vid", "layout_rev", "bases")

    def identical(q):
        k = q.pool_index
        r = q.result
        return r is not None and r["status"] == 0 and all(
            np.array_equal(r[f].astype(np.int64), wants[k][f].astype(np.int64)) for f in fields)

    def measure(resident):
        """Alone service, then the arrival rate for a device-busy fraction of
        about 0.8 and the latency and throughput of that stream.  resident:
        the pool is uploaded once and requests hold only outputs; else every
        request uploads its graph when admitted."""
        tag = "resident" if resident else "upload"

        def mk(lanes, max_wave):
            srv = serve.Server(serve.Device(lanes=lanes, lane_bytes=args.lane_bytes,
                                            max_wave=max_wave))
            if resident:
                for h in pool:
                    srv.make_resident(h)
            return srv

        def stream(n, rate, seed):
            r = np.random.default_rng(seed)
            pick = r.integers(0, n_pool, size=n)
            arr = serve.poisson_arrivals(n, rate, seed + 1) if rate else np.zeros(n)
            out = []
            for i, (k, t) in enumerate(zip(pick, arr)):
                q = serve.Request(i, pool[k], 64, 2, float(t), resident=resident)
                q.pool_index = int(k)
                out.append(q)
            return out

        # each pool graph alone (one lane, waves of one; also the warm-up)
        srv1 = mk(1, 1)
        alone_reqs = []
        for i, h in enumerate(pool):
            q = serve.Request(i, h, 64, 2, 0.0, resident=resident)
            q.pool_index = i
            alone_reqs.append(q)
        alone, _, _, iv = srv1.run(alone_reqs)
        srv1.close()
        del srv1
        svc = np.array([q.t_done - q.t_admit for q in alone])
        dev_alone = sum(i[1] - i[0] for i in iv) / len(alone)
        rate = 0.8 / dev_alone
        log("%s, alone: mean service %.2f ms, device %.3f ms per request -> start rate %.0f/s"
            % (tag, 1e3 * svc.mean(), 1e3 * dev_alone, rate))
        srv = mk(2, args.max_wave)
        n_warm = max(args.requests // 10, 10)
        # search on the arrival rate for a device-busy fraction of about 0.8:
        # proportional steps (at most x4) until the target is bracketed, then
        # bisection; when busy stops rising with the rate the loop is
        # saturated (the host, not the device, sets the pace) and the
        # saturated run is reported.  Otherwise the run closest to 0.8 is.
        lo = hi = None
        best = None
        saturated = False
        trail = []
        for attempt in range(8):
            reqs, span, peak, iv = srv.run(stream(n_warm + args.requests, rate,
                                                  20220709 + attempt))
            busy = serve.busy_fraction(iv, span)
            kbusy = serve.busy_fraction(iv, span, ("kernels",))
            waves = len({q.wave for q in reqs if q.wave is not None})
            log("%s, rate %.0f/s: device busy %.2f (kernels %.2f) over %.2fs, %d waves"
                % (tag, rate, busy, kbusy, span, waves))
            trail.append((rate, busy))
            if best is None or abs(busy - 0.8) < abs(best[0] - 0.8):
                best = (busy, rate, reqs, span, peak, waves, kbusy)
            if abs(busy - 0.8) <= 0.03:
                break
            if busy < 0.8:
                if lo is not None and rate >= 4 * lo and busy < 1.1 * lo_busy:
                    saturated = True
                    break
                lo, lo_busy = rate, busy
            else:
                hi = rate
            rate = 0.5 * (lo + hi) if lo is not None and hi is not None \
                else rate * min(4.0, 0.8 / max(busy, 0.05))
        busy, rate, reqs, span, peak, waves, kbusy = best
        meas = sorted(reqs, key=lambda q: q.rid)[n_warm:]
        failed = [q for q in meas if q.result is None]
        ok = [q for q in meas if q.result is not None]
        lat = np.array([q.t_done - q.arrival for q in ok])
        bases = sum(int(q.result["len"].sum()) for q in ok)
        t_span = max(q.t_done for q in meas) - min(q.arrival for q in meas)
        same = sum(identical(q) for q in meas)
        log("%s: parity %d / %d identical to the oracle" % (tag, same, len(meas)))
        out = {"value": bases / t_span, "unit": "contig bases/s",
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "device_busy_fraction": busy, "kernel_busy_fraction": kbusy,
               "rate_per_s": rate, "requests": len(meas),
               "saturated": saturated,
               "rate_search": [[float(r), float(b)] for r, b in trail],
               "failed_requests": len(failed), "waves": waves,
               "mean_wave_requests": (n_warm + args.requests) / max(waves, 1),
               "warmup_requests": n_warm, "lanes": 2, "max_wave": args.max_wave,
               "lane_bytes": args.lane_bytes, "budget_bytes": srv.budget,
               "peak_admitted_bytes": int(peak),
               "parity": {"identical": int(same), "total": len(meas)},
               "alone_service_ms": {"mean": float(svc.mean() * 1e3),
                                    "max": float(svc.max() * 1e3)},
               "alone_device_ms_per_request": dev_alone * 1e3}
        srv.close()
        return out

    upload = measure(False)
    res = measure(True)
    result = {
        "metric": "contig bases/s (serving, continuous batching)",
        "value": res["value"],
        "unit": "contig bases/s",
        "n_gpus": 1,
        "higher_is_better": True,
    }
    result.update({k: v for k, v in res.items() if k not in ("value", "unit")})
    result.update({
        "with_upload": upload,
        "dtype": "int32",
        "data": "synthetic (seeded simulated genomes and reads; exact reduced string graphs)",
        "config": {"workload": "serving: Poisson stream over a pool of %d request graphs (genome "
                               "1-100 Mbp log-uniform, 15-30x, reads LN(12k, 4k), 1-2%% branch "
                               "edges, P = 64)" % n_pool,
                   "resident": "the pool's graphs are resident in HBM (uploaded once, before "
                               "the stream); each wave of admitted requests is planned into a "
                               "lane's batch and run as one batched launch sequence, and its "
                               "contigs are packed by the library and downloaded in one copy",
                   "latency": "arrival to contigs in pinned host memory (all five steps and "
                              "the download; with_upload: the graph's upload and check as "
                              "well)",
                   "device_busy": "union of the GPU-event intervals of every wave's kernels "
                                  "(batched path, result packing) and result download, over "
                                  "the run's span; kernel_busy_fraction: the kernels alone"},
    })
    if not args.no_cpu:
        graphs = [h.graph for h in pool]
        cbases = sum(int(w["len"].sum()) for w in wants)
        passes = 1
        while spent < min(MIN_CPU_SECONDS, args.cpu_seconds):
            for g in graphs:
                tm = {}
                cbases += int(oracle.run(g, P=64, min_reads=2, timings=tm)["contigs"]["len"].sum())
                spent += tm["total"]
            passes += 1
        result["cpu_baseline"] = {
            "value": cbases / spent, "unit": "contig bases/s", "cores": 1, "kind": "oracle",
            "sample": "%d pass(es) over the %d request graphs of the pool, single-threaded C "
                      "oracle, whole path (no uploads)" % (passes, n_pool),
            "seconds": spent}
        result["host"] = host_info()
        if args.cpu_workers > 1:
            result["cpu_baseline_pool"] = cpu_pool_baseline(graphs, [64] * n_pool,
                                                            args.cpu_workers,
                                                            src=("request", n_pool))
            log("oracle pool: %d processes, %.2fs" % (args.cpu_workers,
                                                      result["cpu_baseline_pool"]["seconds"]))
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()

"""Launch-shape tuner for the batched form.

Tries candidate cg_batch_params on the actual batch, times each launch of
each candidate's captured HIP graph, and keeps the one with the smallest
median.  Every candidate's outputs are compared, array by array on the
device, with the first candidate's: a shape may change speed, never a byte
of the result.  Results are cached per batch shape (number of jobs, reads,
entries) in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

from . import cg

VERTEX_TILES = (256, 512, 1024)
COPY_BLOCKS = (64, 256, 512)
PERSIST = (512, 1024, 2048)

_CACHE = os.environ.get("CG_TUNE_CACHE",
                        os.path.join(os.path.expanduser("~"), ".cache", "cg_batch_tune.json"))


def _key(jobs):
    n = sum(job[0].n for job in jobs)
    m = sum(job[0].m for job in jobs)
    return "%d:%d:%d" % (len(jobs), n, m)


def _snapshot(jobs):
    """Device copies of every output that defines the result."""
    snap = []
    for job in jobs:
        dg, out = job[0], job[1]
        nc = int(out.n_comp.item())
        ne = int(out.sizes[0].item())
        me = int(out.sizes[1].item())
        tw = int(out.total_words.item())
        snap.append([t.clone() for t in (
            out.flags[:dg.n], out.counts, out.label[:dg.n], out.comp_label[:nc],
            out.comp_size[:nc], out.comp_kind[:nc], out.comp_bin[:nc], out.comp_rank[:nc],
            out.comp_start[:nc], out.bin_load, out.label_comp[:dg.n], out.perm[:ne],
            out.bin_vptr, out.loc_row_ptr[:ne + 1], out.loc_col[:me], out.loc_eid[:me],
            out.c_label[:nc], out.c_bin[:nc], out.c_start[:nc], out.c_nreads[:nc],
            out.c_len[:nc], out.c_base_off[:nc], out.c_flags[:nc], out.c_layout_off[:nc],
            out.layout_vid[:ne], out.layout_rev[:ne], out.bases[:tw], out.total_words)])
    return snap


def _same(snap, jobs):
    import torch
    cur = _snapshot(jobs)
    return all(a.shape == b.shape and torch.equal(a, b)
               for sa, sb in zip(snap, cur) for a, b in zip(sa, sb))


def tune(ctx, jobs, stream, reps=10, candidates=None, use_cache=True, log=None):
    """Return (best (vertex_tile, copy_block, persist_blocks), {shape: ms})."""
    import torch
    key = _key(jobs)
    cache = {}
    if use_cache and os.path.exists(_CACHE):
        try:
            cache = json.load(open(_CACHE))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return tuple(cache[key]["best"]), cache[key]["table"]
    if candidates is None:
        candidates = [(v, c, p) for v in VERTEX_TILES for c in COPY_BLOCKS for p in PERSIST]
    table = {}
    ref = None
    best, best_ms = None, float("inf")
    for shape in candidates:
        b = cg.Batch(ctx, jobs, *shape)
        with torch.cuda.stream(stream):
            b.capture(stream)
            b.launch(stream)
        stream.synchronize()
        if ref is None:
            ref = _snapshot(jobs)
        elif not _same(ref, jobs):
            raise RuntimeError("launch shape %s changed the result" % (shape,))
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        with torch.cuda.stream(stream):
            b.launch(stream)  # warm
            ev[0].record(stream)
            for i in range(reps):
                b.launch(stream)
                ev[i + 1].record(stream)
        stream.synchronize()
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(reps))[reps // 2]
        table["%d/%d/%d" % shape] = ms
        if log:
            log("tune %s: %.3f ms" % (shape, ms))
        if ms < best_ms:
            best, best_ms = shape, ms
        b.close()
    if use_cache:
        cache[key] = {"best": list(best), "table": table, "when": time.time()}
        try:
            os.makedirs(os.path.dirname(_CACHE), exist_ok=True)
            json.dump(cache, open(_CACHE, "w"))
        except OSError:
            pass
    return best, table

"""GPU parity of the batched form: every job of a batch equals the oracle on
that graph, for every launch shape, eagerly and replayed from a HIP graph."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.parity import mismatches
from tests.test_gpu_parity import _chain_graph

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_04350_amd import cg as _cg
    _cg.lib()
    return _cg


def _mixed_graphs():
    rng = np.random.default_rng(17)
    gs = [synth.adversarial(rng) for _ in range(40)]
    gs.append(synth.graph_from_edges([], []))                       # empty graph
    gs.append(synth.config_graph(1))
    gs += synth.batch_graphs(only=[0, 7, 300])
    r = np.random.default_rng(5)
    gs.append(_chain_graph(r, [1500, 40, 2], cycles=[1200, 7]))   # beyond the LDS tiles
    gs.append(_chain_graph(r, [2] * 2500 + [5] * 30))              # beyond the batch LDS sort
    gs.append(_chain_graph(r, [3000, 2900, 2400, 3]))
    # explicit alignment coordinates: x-drop clips, and arbitrary values
    from tests.test_oracle_overhangs import _random_pre_post
    gs.append(synth.with_alignment_ends(synth.config_graph(1), np.random.default_rng(8), 3))
    ra = np.random.default_rng(18)
    gs += [_random_pre_post(synth.adversarial(ra), ra) for _ in range(6)]
    # more entries than the batched components pass takes: run through the
    # single-graph kernels inside the batch, with and without one-read
    # components
    gs.append(_chain_graph(r, [6000, 6000, 5000, 2]))
    gs[-1].meta["min_reads"] = 2
    gs.append(_chain_graph(r, [7000, 5000, 1], cycles=[4000, 600]))
    gs[-1].meta["min_reads"] = 1
    # explicit coordinates through every batched walk form: one-wave walks
    # (up to 128 reads), the one-pass LDS walk (129-512) and the two-pass
    # global-array walk (above 512: the induce step's sort in LDS up to 1024
    # reads, in scratch above), chains and cycles, clipped and arbitrary;
    # and a job with coordinates above the batched entry bound (single-graph
    # route)
    rc = np.random.default_rng(33)
    gs.append(synth.with_alignment_ends(
        _chain_graph(rc, [128, 129, 512, 513, 1024, 1025], cycles=[512, 513, 1024],
                     len_lo=30, len_hi=80), rc, 3))
    gs[-1].meta = dict(gs[-1].meta, min_reads=2)
    gs.append(synth.with_alignment_ends(
        _chain_graph(rc, [200, 900, 3000, 60], cycles=[1500], len_lo=30, len_hi=80), rc, 3))
    gs[-1].meta = dict(gs[-1].meta, min_reads=2)
    gs.append(_random_pre_post(
        _chain_graph(rc, [1500, 2], cycles=[200, 900, 3000], len_lo=30, len_hi=80), rc))
    gs[-1].meta = dict(min_reads=1)
    gs.append(synth.with_alignment_ends(_chain_graph(rc, [6000, 5000, 4000, 2000, 500, 2],
                                                     cycles=[1200], len_lo=30, len_hi=80),
                                        rc, 3))
    gs[-1].meta = dict(gs[-1].meta, min_reads=2)
    # more listed reads than the components pass holds in LDS, but few
    # entries: the components pass keeps their state in the job's scratch
    gs.append(_chain_graph(r, [2] * 9000))
    gs[-1].meta["min_reads"] = 2
    gs.append(_chain_graph(r, [2] * 8800 + [3] * 50))
    gs[-1].meta["min_reads"] = 1
    return gs


def _params(i, g):
    """(P, min_reads, weight) of job i: every third job partitions by bases."""
    w = "bases" if i % 3 == 1 else "reads"
    if "min_reads" in g.meta:
        return [64, 300, 8, 1024][i % 4], g.meta["min_reads"], w
    r = np.random.default_rng(100 + i)
    P = int(r.integers(1, 9)) if g.n <= 16 else [64, 300, 8, 1024][i % 4]
    return P, int(r.integers(0, 3)) if g.n <= 16 else 2, w


def _make(cg, graphs, params, **shape):
    import torch
    dev = torch.device("cuda")
    big = max(range(len(graphs)), key=lambda i: cg.footprint(graphs[i].n, graphs[i].m,
                                                             params[i][0]))
    ctx = cg.Context.for_graph(graphs[big].n, graphs[big].m, params[big][0])
    dgs = [cg.DeviceGraph(g, dev) for g in graphs]
    outs = [cg.Outputs(g.n, p[0], g.seq_words, dev) for g, p in zip(graphs, params)]
    b = cg.Batch(ctx, [(dg, o) + tuple(p) for dg, o, p in zip(dgs, outs, params)], **shape)
    return ctx, dgs, outs, b


def _scrub(outs):
    for o in outs:
        for t in (o.flags, o.label, o.comp_label, o.comp_bin, o.comp_start, o.perm,
                  o.loc_col, o.layout_vid, o.c_len, o.c_base_off, o.bases, o.n_comp,
                  o.total_words, o.sizes):
            t.fill_(-1 if t.dtype != __import__("torch").uint8 else 255)


def _explain_bases(got, want):
    a, b = got["contigs"]["bases"], want["contigs"]["bases"]
    if a.shape != b.shape:
        return "shape %s vs %s" % (a.shape, b.shape)
    d = np.nonzero(a != b)[0]
    c = want["contigs"]
    words = (c["base_off"] // 16).astype(np.int64)
    out = []
    for w in d[:4]:
        k = int(np.searchsorted(words, w, side="right") - 1)
        out.append("word %d got %08x want %08x contig %d (len %d, words %d..%d, n_reads %d)" % (
            w, a[w], b[w], k, c["len"][k], words[k], words[k] + (int(c["len"][k]) + 15) // 16,
            c["n_reads"][k]))
    return "%d words differ; " % len(d) + "; ".join(out)


def _check_all(cg, graphs, params, outs, wants, tag):
    for i, (g, o) in enumerate(zip(graphs, outs)):
        got = cg.to_host(o, g.n)
        bad = mismatches(got, wants[i])
        if bad == ["contigs.bases"]:
            _say("bases mismatch", tag, i, _explain_bases(got, wants[i]))
        assert bad == [], (tag, i, g.meta.get("name"), bad)


def test_batch_mixed_all_shapes(cg):
    import torch
    graphs = _mixed_graphs()
    params = [_params(i, g) for i, g in enumerate(graphs)]
    wants = [oracle.run(g, P=P, min_reads=mr, weight=w) for g, (P, mr, w) in zip(graphs, params)]
    for shape in (dict(), dict(vertex_tile=512, copy_block=128, persist_blocks=64),
                  dict(vertex_tile=1024, copy_block=1024, persist_blocks=7),
                  dict(vertex_tile=256, copy_block=64, persist_blocks=2048)):
        _say("batch shape", shape, "jobs", len(graphs))
        ctx, dgs, outs, b = _make(cg, graphs, params, **shape)
        b.run()
        torch.cuda.synchronize()
        assert ctx.status() == 0
        _check_all(cg, graphs, params, outs, wants, "eager %s" % shape)
        # the launch state resets itself: a second run gives the same result
        _scrub(outs)
        b.run()
        torch.cuda.synchronize()
        _check_all(cg, graphs, params, outs, wants, "rerun %s" % shape)
        b.close()
        ctx.close()


def test_batch_graph_replay(cg):
    import torch
    graphs = _mixed_graphs()[30:]
    params = [_params(i, g) for i, g in enumerate(graphs)]
    wants = [oracle.run(g, P=P, min_reads=mr, weight=w) for g, (P, mr, w) in zip(graphs, params)]
    ctx, dgs, outs, b = _make(cg, graphs, params)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(s)
    s.synchronize()
    _check_all(cg, graphs, params, outs, wants, "eager")
    with torch.cuda.stream(s):
        b.capture(s)
    for rep in range(4):
        _say("replay", rep)
        _scrub(outs)                       # eager work between replays
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.launch(s)
        s.synchronize()
        assert ctx.status(s) == 0
        _check_all(cg, graphs, params, outs, wants, "replay %d" % rep)
    b.close()
    ctx.close()


def test_batch_512_graphs(cg):
    """The batched workload in full: 512 graphs in one batch."""
    import torch
    graphs = synth.batch_graphs(512)
    params = [(g.meta["P"], 2, "bases" if i % 2 else "reads") for i, g in enumerate(graphs)]
    ctx, dgs, outs, b = _make(cg, graphs, params)
    b.run()
    torch.cuda.synchronize()
    for i, g in enumerate(graphs):
        want = oracle.run(g, P=params[i][0], min_reads=2, weight=params[i][2])
        got = cg.to_host(outs[i], g.n)
        bad = mismatches(got, want)
        if bad == ["contigs.bases"]:
            _say("bases mismatch job", i, _explain_bases(got, want))
        assert bad == [], (i, bad)
    b.close()
    ctx.close()


def test_batch_lpt_equal_runs(cg):
    """Runs of equal read counts in the batched LPT (rounds with at most 64
    bins), in LDS and beyond it (more than 2048 components)."""
    import torch
    rng = np.random.default_rng(9)
    graphs = [_chain_graph(rng, [int(x) for x in rng.permutation(
        [6] * 60 + [3] * 400 + [2] * 900)]) for _ in range(3)]
    graphs.append(_chain_graph(rng, [int(x) for x in rng.permutation([4] * 300 + [2] * 2500)]))
    params = [(P, 2, "reads") for P in (1, 7, 64, 33)]
    wants = [oracle.run(g, P=P, min_reads=mr, weight=w) for g, (P, mr, w) in zip(graphs, params)]
    _say("batch equal runs", [g.n for g in graphs])
    ctx, dgs, outs, b = _make(cg, graphs, params)
    b.run()
    torch.cuda.synchronize()
    assert ctx.status() == 0
    _check_all(cg, graphs, params, outs, wants, "equal runs")
    b.close()
    ctx.close()


def test_batch_replan(cg):
    """One batch's memory planned with one job set after another (as a
    serving loop does): each run equals the oracle, and a plan beyond the
    batch's memory is refused without touching it."""
    import torch
    graphs = _mixed_graphs()
    sets = [list(range(0, 20)), list(range(40, 52)), list(range(20, 45)), list(range(0, 20))]
    params = [_params(i, g) for i, g in enumerate(graphs)]
    wants = {}
    dev = torch.device("cuda")
    big = max(range(len(graphs)), key=lambda i: cg.footprint(graphs[i].n, graphs[i].m,
                                                             params[i][0]))
    ctx = cg.Context.for_graph(graphs[big].n, graphs[big].m, params[big][0])
    dgs = {}
    jobs_of = {}
    for sel in sets:
        for i in sel:
            if i not in dgs:
                dgs[i] = cg.DeviceGraph(graphs[i], dev)
    cap = 0
    for k, sel in enumerate(sets):
        outs = [cg.Outputs(graphs[i].n, params[i][0], graphs[i].seq_words, dev) for i in sel]
        jobs_of[k] = [(dgs[i], o) + tuple(params[i]) for i, o in zip(sel, outs)]
        cap = max(cap, cg.batch_bytes(jobs_of[k]))
    b = cg.Batch.empty(ctx, cap)
    s = torch.cuda.Stream()
    for k, sel in enumerate(sets):
        _say("replan", k, "jobs", len(sel))
        with torch.cuda.stream(s):
            b.plan(jobs_of[k], s)
            b.run(s)
        s.synchronize()
        assert ctx.status(s) == 0
        for i, job in zip(sel, jobs_of[k]):
            if i not in wants:
                P, mr, w = params[i]
                wants[i] = oracle.run(graphs[i], P=P, min_reads=mr, weight=w)
            got = cg.to_host(job[1], graphs[i].n)
            bad = mismatches(got, wants[i])
            assert bad == [], ("replan", k, i, bad)
    small = cg.Batch.empty(ctx, 4096)
    with pytest.raises(cg.CgError) as e:
        small.plan(jobs_of[1], s)
    assert e.value.code == cg.CG_ECAPACITY
    small.close()
    b.close()
    ctx.close()


def test_batch_carved_outputs_and_packed_results(cg):
    """Outputs carved from one buffer per batch (cg_job_outputs), results
    counted (cg_batch_counts) and packed (cg_batch_pack) into one buffer:
    every job's unpacked records, layout and bases equal the oracle, the
    offsets tile the packed buffer, and nothing is written past dst_bytes."""
    import torch
    graphs = _mixed_graphs()
    params = [_params(i, g) for i, g in enumerate(graphs)]
    dev = torch.device("cuda")
    ctx = cg.Context(0, 0)
    dgs = [cg.DeviceGraph(g, dev) for g in graphs]
    sizes = [cg.job_outputs_bytes(g.n, p[0], g.seq_words) for g, p in zip(graphs, params)]
    buf = torch.full((sum(sizes),), 0xA5, dtype=torch.uint8, device=dev)
    outs, at = [], 0
    for g, p, nb in zip(graphs, params, sizes):
        outs.append(cg.CarvedOutputs(buf, at, g.n, p[0], g.seq_words))
        at += nb
    jobs = [(dg, o) + tuple(p) for dg, o, p in zip(dgs, outs, params)]
    b = cg.Batch.empty(ctx, cg.batch_bytes(jobs))
    s = torch.cuda.Stream()
    _say("carved batch", len(jobs))
    with torch.cuda.stream(s):
        b.plan(jobs, s)
        b.run(s)
        d_counts = torch.empty(4 * len(jobs) + 1, dtype=torch.int64, device=dev)
        b.counts(d_counts, s)
    s.synchronize()
    assert ctx.status(s) == 0
    counts = d_counts.cpu().numpy()
    rows = counts[:-1].reshape(-1, 4)
    total = int(counts[-1])
    assert total % 16 == 0 and rows[0, 3] == 0
    assert np.all(rows[:, 3] % 16 == 0)
    ends = rows[:, 3] + ((40 * rows[:, 0] + 5 * rows[:, 1] + 4 * rows[:, 2] + 15) // 16) * 16
    assert np.array_equal(ends[:-1], rows[1:, 3]) and ends[-1] == total
    # packed into a buffer with a guard band that must stay untouched
    dst = torch.full((total + 4096,), 0x5A, dtype=torch.uint8, device=dev)
    with torch.cuda.stream(s):
        b.pack(d_counts, dst[:total], s)
    s.synchronize()
    packed = dst.cpu().numpy()
    assert np.all(packed[total:] == 0x5A)
    for i, (g, p) in enumerate(zip(graphs, params)):
        want = oracle.run(g, P=p[0], min_reads=p[1], weight=p[2])["contigs"]
        got = cg.unpack_results(packed, rows[i])
        assert rows[i][0] == want["label"].shape[0], i
        assert rows[i][2] == want["total_words"], i
        for name in ("label", "bin", "start", "n_reads", "len", "base_off", "cflags",
                     "layout_off", "layout_vid", "layout_rev", "bases"):
            assert np.array_equal(got[name].astype(np.int64), want[name].astype(np.int64)), \
                (i, name)
    # a short destination: the copy stops at dst_bytes
    half = (total // 2) & ~15
    dst.fill_(0x5A)
    with torch.cuda.stream(s):
        b.pack(d_counts, dst[:half], s)
    s.synchronize()
    short = dst.cpu().numpy()
    assert np.array_equal(short[:half], packed[:half]) and np.all(short[half:] == 0x5A)
    b.close()
    ctx.close()

"""GPU parity: every output of the five C-ABI calls equals the oracle's,
element by element (all outputs are integers or packed bases: exact)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.parity import mismatches

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


def run_gpu(cg, g, P, min_reads=2, ctx=None, cap_words=None, weight="reads"):
    own = ctx is None
    if own:
        ctx = cg.Context.for_graph(g.n, g.m, P)
    dg = cg.DeviceGraph(g, "cuda")
    out = cg.Outputs(g.n, P, g.seq_words if cap_words is None else cap_words, "cuda")
    cg.run_path(ctx, dg, out, P, min_reads, weight=weight)
    got = cg.to_host(out, g.n)
    if own:
        ctx.close()
    return got, out


def check(cg, g, P, min_reads=2, ctx=None, name="", weight="reads"):
    _say("parity case", name, "n=%d m=%d P=%d min_reads=%d weight=%s" % (g.n, g.m, P, min_reads,
                                                                          weight))
    got, _ = run_gpu(cg, g, P, min_reads, ctx, weight=weight)
    want = oracle.run(g, P=P, min_reads=min_reads, weight=weight)
    bad = mismatches(got, want)
    assert bad == [], (name, bad)
    return got


def test_paper_examples(cg, golden):
    ex = golden["masking"]
    reads = [np.zeros(20, np.uint8) for _ in range(8)]
    g = synth.graph_from_edges(reads, [(a, b, 5, 0, 0) for a, b in ex["edges"]])
    for P in (1, 2, 3, 8):
        check(cg, g, P, 2, name="masking-P%d" % P)
    c = golden["concatenation"]
    g = synth.graph_from_edges([synth.encode(s) for s in c["reads"]],
                               [(0, 1, 4, 0, 0), (1, 2, 5, 0, 0)])
    check(cg, g, 1, 2, name="fig3")
    r = golden["reverse_strand"]
    g = synth.graph_from_edges([synth.encode(s) for s in r["reads"]],
                               [(0, 1, 4, 0, 1), (1, 2, 5, 1, 0)])
    got = check(cg, g, 1, 2, name="fig3-reverse")
    L = int(got["contigs"]["len"][0])
    assert synth.decode(oracle.contig_codes(got["contigs"], 0)) == r["contig"]
    assert L == len(r["contig"])


def test_adversarial_corpus(cg):
    rng = np.random.default_rng(7)
    graphs = [synth.adversarial(rng) for _ in range(300)]
    ctx = cg.Context.for_graph(16, 64, 8)
    for i, g in enumerate(graphs):
        r = np.random.default_rng(1000 + i)
        P = int(r.integers(1, 9))
        mr = int(r.integers(0, 3))
        check(cg, g, P, mr, ctx=ctx, name="adversarial-%d" % i)
    ctx.close()


@pytest.mark.parametrize("cfg", [1, 2])
def test_config_full(cg, cfg):
    g = synth.config_graph(cfg)
    check(cg, g, g.meta["P"], 2, name="config%d" % cfg)


def test_config3_full(cg):
    g = synth.config_graph(3)
    check(cg, g, g.meta["P"], 2, name="config3")
    # the most bins there can be: 231k contig reads need more than the 16 load
    # bits a 32-bit key leaves, so the LPT takes its 64-bit keys
    check(cg, g, 65536, 2, name="config3-P65536")


def test_batch_and_request_graphs(cg):
    gs = synth.batch_graphs(only=[0, 1, 2, 3, 100, 511])
    rp = synth.request_params(40)
    small = sorted(range(40), key=lambda i: rp[i]["G"])[:3]
    gs += [synth.simulate(**rp[i]) for i in small]
    for g in gs:
        check(cg, g, g.meta["P"], 2, name=g.meta["name"])


def test_empty_and_tiny(cg):
    g0 = synth.graph_from_edges([], [])
    check(cg, g0, 4, 2, name="empty")
    g1 = synth.graph_from_edges([synth.encode("ACGT")], [])
    check(cg, g1, 4, 1, name="single-read-min1")
    check(cg, g1, 4, 2, name="single-read-min2")
    # a star: the centre is a branch vertex, its leaves become single reads
    reads = [synth.encode("ACGTACGTAC") for _ in range(5)]
    g = synth.graph_from_edges(reads, [(0, i, 3, 0, 0) for i in range(1, 5)])
    check(cg, g, 3, 1, name="star")
    check(cg, g, 3, 2, name="star-min2")


def _chain_graph(rng, sizes, cycles=(), len_lo=8, len_hi=40):
    """Disjoint chains (and cycles) over randomly numbered reads."""
    n = int(sum(sizes) + sum(cycles))
    ids = rng.permutation(n)
    lens = rng.integers(len_lo, len_hi + 1, size=n)
    reads = [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in lens]
    edges = []
    at = 0
    for q, cyc in [(q, False) for q in sizes] + [(q, True) for q in cycles]:
        grp = ids[at:at + q]
        at += q
        pairs = list(zip(grp[:-1], grp[1:])) + ([(grp[-1], grp[0])] if cyc else [])
        for a, b in pairs:
            hi = int(min(lens[a], lens[b])) - 1
            edges.append((int(a), int(b), int(rng.integers(1, hi + 1)), int(rng.integers(0, 2)),
                          int(rng.integers(0, 2))))
    return synth.graph_from_edges(reads, edges)


def test_components_beyond_lds(cg):
    """Chains and cycles longer than the per-component LDS tiles."""
    rng = np.random.default_rng(5)
    g = _chain_graph(rng, [3000, 1025, 2, 700], cycles=[2500, 1100, 5])
    check(cg, g, 3, 2, name="long-chains")


def test_many_components_and_bins(cg):
    rng = np.random.default_rng(6)
    g = _chain_graph(rng, [2] * 9000 + [3] * 200 + [17] * 50)
    check(cg, g, 64, 2, name="9250-components")      # beyond the LDS sort
    check(cg, g, 3000, 2, name="3000-bins")          # beyond the LDS bin list
    g2 = _chain_graph(rng, list(rng.integers(2, 60, size=3000)))
    for P in (65, 200, 1024, 5000):
        check(cg, g2, P, 2, name="windows-P%d" % P)  # windowed LPT with merges


def test_lpt_equal_runs(cg):
    """Long runs of components with equal read counts: with at most 64 bins
    the LPT places such runs in rounds; the partition must stay the one the
    oracle's component-by-component LPT gives."""
    rng = np.random.default_rng(8)
    sizes = [9] * 40 + [5] * 300 + [4] * 500 + [3] * 7 + [2] * 1200
    g = _chain_graph(rng, [int(x) for x in rng.permutation(sizes)])
    for P in (1, 7, 33, 64):
        check(cg, g, P, 2, name="equal-runs-P%d" % P)


def test_lpt_prefix_rounds(cg):
    """Components of many different read counts: the LPT places runs of
    items whose bins stay the least loaded in one round (prefix rounds), with
    and without windows of bins; the partition must stay the oracle's."""
    rng = np.random.default_rng(9)
    cases = [
        ("spread", [int(x) for x in rng.integers(2, 400, size=700)]),
        ("pow2", [int(2 ** x) for x in rng.integers(1, 9, size=500)]),
        ("consecutive", list(range(2, 302))),
        ("few-large", [300, 299, 298] + [int(x) for x in rng.integers(2, 6, size=900)]),
    ]
    for name, sizes in cases:
        g = _chain_graph(rng, [int(x) for x in rng.permutation(sizes)])
        for P in (2, 8, 63, 64, 100, 1024):
            check(cg, g, P, 2, name="prefix-%s-P%d" % (name, P))


def test_lpt_many_components(cg):
    """More components than the LPT sorts hold in LDS (8192), with 32-bit
    keys (fewer than 65536 components) and with 64-bit keys (more)."""
    rng = np.random.default_rng(10)
    for name, sizes in (("20k", [2] * 15000 + [int(x) for x in rng.integers(3, 40, size=5000)]),
                        ("70k", [2] * 66000 + [int(x) for x in rng.integers(3, 9, size=4000)])):
        g = _chain_graph(rng, [int(x) for x in rng.permutation(sizes)], len_lo=20, len_hi=30)
        for P in (7, 64, 1024):
            check(cg, g, P, 2, name="many-%s-P%d" % (name, P))


def test_deterministic(cg):
    g = synth.config_graph(2)
    P = g.meta["P"]
    a, _ = run_gpu(cg, g, P)
    b, _ = run_gpu(cg, g, P)
    assert mismatches(a, b) == []


def test_capacity_overflow(cg):
    import torch
    g = synth.config_graph(1)
    P = g.meta["P"]
    want = oracle.run(g, P=P)
    need = want["contigs"]["total_words"]
    ctx = cg.Context.for_graph(g.n, g.m, P)
    dg = cg.DeviceGraph(g, "cuda")
    out = cg.Outputs(g.n, P, need - 1, "cuda")
    out.bases.fill_(0x5A5A5A5A)
    cg.run_path(ctx, dg, out, P, 2)
    torch.cuda.synchronize()
    assert int(out.total_words.item()) == need
    assert (out.bases.cpu().numpy() == 0x5A5A5A5A).all()
    assert ctx.status() & cg.STATUS_BASES_OVERFLOW
    assert ctx.status() == 0   # cleared by the previous read
    ctx.close()


def test_validate_matches_oracle(cg):
    import torch
    from tests.test_oracle_pins import NEGATIVE, break_graph
    reads = [np.zeros(10, np.uint8) for _ in range(4)]
    ctx = cg.Context.for_graph(8, 8, 1)
    for case in [None] + sorted(NEGATIVE):
        g = synth.graph_from_edges(reads, [(0, 1, 3, 0, 0), (1, 2, 3, 1, 0)])
        if case is not None:
            g = break_graph(g, case)
        _say("validate case", case)
        dg = cg.DeviceGraph(g, "cuda")
        bad = torch.empty(2, dtype=torch.int64, device="cuda")
        cg.validate(ctx, dg, bad)
        got = tuple(int(x) for x in bad.cpu().numpy())
        assert got == oracle.validate(g), case
    ctx.close()


def test_alignment_ends(cg):
    """Explicit per-entry (pre, post) (Section 4.4): consistent x-drop clips
    on reads with errors, and arbitrary in-range values (empty pieces,
    same-end joins) on the adversarial corpus."""
    from tests.test_oracle_overhangs import _random_pre_post
    g = synth.with_alignment_ends(synth.config_graph(1), np.random.default_rng(4), max_clip=3)
    check(cg, g, 8, 2, name="config1-clipped")
    check(cg, g, 3, 1, name="config1-clipped-singles")
    rng = np.random.default_rng(12)
    ctx = cg.Context.for_graph(64, 256, 16)
    for i in range(150):
        h = _random_pre_post(synth.adversarial(rng), rng)
        P, mr = int(rng.integers(1, 9)), int(rng.integers(0, 3))
        got, _ = run_gpu(cg, h, P, mr, ctx)
        bad = mismatches(got, oracle.run(h, P=P, min_reads=mr))
        assert bad == [], (i, bad)
    ctx.close()


def test_alignment_ends_long_components(cg):
    """Explicit (pre, post) through every walk form: components of 200 and
    900 reads (the LDS walk of one workgroup) and of 1,500 and 3,000 reads
    (the walk over global arrays), as chains and as cycles, with consistent
    x-drop clips and with arbitrary in-range coordinates (Section 4.4); and
    the 50 Mbp workload with clips."""
    from tests.test_oracle_overhangs import _random_pre_post
    rng = np.random.default_rng(31)
    g = _chain_graph(rng, [200, 900, 1500, 3000, 2], cycles=[200, 900, 1500, 3000],
                     len_lo=30, len_hi=80)
    check(cg, synth.with_alignment_ends(g, rng, max_clip=3), 4, 2, name="long-clipped")
    check(cg, _random_pre_post(g, rng), 4, 2, name="long-random-coords")
    check(cg, _random_pre_post(g, rng), 3, 1, name="long-random-coords-min1")
    g2 = synth.with_alignment_ends(synth.config_graph(2), np.random.default_rng(32), max_clip=3)
    check(cg, g2, 64, 2, name="config2-clipped")


def test_bases_weighted_partition(cg):
    """GreedyPartitioning by bases (the total read length of a component)."""
    check(cg, synth.config_graph(1), 8, 2, name="config1-bases", weight="bases")
    check(cg, synth.config_graph(2), 64, 2, name="config2-bases", weight="bases")
    check(cg, synth.config_graph(2), 3000, 2, name="config2-bases-3000-bins", weight="bases")
    rng = np.random.default_rng(21)
    ctx = cg.Context.for_graph(64, 256, 16)
    for i in range(150):
        g = synth.adversarial(rng)
        P, mr = int(rng.integers(1, 9)), int(rng.integers(0, 3))
        got, _ = run_gpu(cg, g, P, mr, ctx, weight="bases")
        bad = mismatches(got, oracle.run(g, P=P, min_reads=mr, weight="bases"))
        assert bad == [], (i, bad)
    ctx.close()

"""GPU parity of cg_reduce (contained-read pruning and transitive reduction
of an overlap graph, Algorithm 1) with the oracle: contained flags, kept
entries and the string graph, element by element (integers: exact)."""
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


def reduce_gpu(cg, r, fuzz=0, ctx=None):
    own = ctx is None
    if own:
        ctx = cg.Context.for_graph(r.n, r.m, 1)
    dg = cg.DeviceGraph(r, "cuda")
    out = cg.Reduced(r.n, r.m, "cuda")
    cg.reduce(ctx, dg, out, fuzz)
    import torch
    torch.cuda.synchronize()
    assert ctx.status() == 0
    m = int(out.d_m.item())
    got = dict(contained=out.contained[:r.n].cpu().numpy(), kept=out.kept[:r.m].cpu().numpy(),
               row_ptr=out.row_ptr.cpu().numpy(), col=out.col[:m].cpu().numpy(),
               ovl=out.ovl[:m].cpu().numpy().view(np.uint32), strand=out.strand[:m].cpu().numpy())
    if own:
        ctx.close()
    return got, out, dg


def check(cg, r, fuzz=0, name=""):
    _say("reduce case", name, "n=%d m=%d fuzz=%d" % (r.n, r.m, fuzz))
    got, out, dg = reduce_gpu(cg, r, fuzz)
    c, k, s = oracle.reduce(r, fuzz=fuzz)
    assert np.array_equal(got["contained"], c), name
    assert np.array_equal(got["kept"], k), name
    for f in ("row_ptr", "col", "ovl", "strand"):
        assert np.array_equal(got[f], getattr(s, f)), (name, f)
    return got, out, dg, s


@pytest.mark.parametrize("seed,G,cov,extra,fuzz", [(31, 300_000, 20, 0.0, 0),
                                                   (32, 1_500_000, 30, 0.02, 0),
                                                   (33, 800_000, 40, 0.01, 3),
                                                   (34, 2_000_000, 12, 0.03, 0)])
def test_generated_overlap_graphs(cg, seed, G, cov, extra, fuzz):
    g = synth.simulate(G=G, cov=cov, mean_len=10_000, sd_len=3_000, err=0.0, extra_rate=extra,
                       seed=seed)
    check(cg, synth.overlap_graph(g), fuzz, name="seed%d" % seed)


def test_row_beyond_lds(cg):
    # a hub read with 1100 neighbours (its row is read in place), each
    # neighbour overlapping the next one: every hub entry but the first is
    # transitive through the previous neighbour
    k = 1100
    rng = np.random.default_rng(1)
    reads = [rng.integers(0, 4, size=100_000).astype(np.uint8)] + \
            [rng.integers(0, 4, size=10_000).astype(np.uint8) for _ in range(k)]
    edges = [(0, i, 10_000 - 5 * i, 0, 0) for i in range(1, k + 1)]
    edges += [(i, i + 1, 9_995, 0, 0) for i in range(1, k)]
    r = synth.graph_from_edges(reads, edges)
    got, out, dg, s = check(cg, r, name="hub")
    assert got["row_ptr"][1] == 1                   # the hub keeps one entry
    assert s.m == 2 * k


def test_path_on_the_reduced_graph(cg):
    g = synth.simulate(G=1_000_000, cov=25, mean_len=10_000, sd_len=3_000, err=0.0,
                       extra_rate=0.02, seed=35)
    r = synth.overlap_graph(g)
    got, out, dg, s = check(cg, r, name="path")
    ctx = cg.Context.for_graph(r.n, r.m, 8)
    sdg = out.graph(dg)
    res = cg.Outputs(r.n, 8, r.seq_words, "cuda")
    cg.run_path(ctx, sdg, res, 8, 2)
    want = oracle.run(s, P=8)
    assert mismatches(cg.to_host(res, r.n), want) == []
    ctx.close()

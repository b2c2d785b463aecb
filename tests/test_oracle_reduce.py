"""Pins of the oracle's step before the path: Prune(IsContainedRead) and
TransitiveReduction (Algorithm 1), with redundant vertices and redundant
edges as Section 2 defines them.

The strongest pin does not go through the oracle's own arithmetic: the
generator builds its string graph directly from the reads' genome intervals
(consecutive non-contained reads), and knows which reads are contained.
Reducing the overlap graph of the same reads must give exactly that graph."""
import dataclasses

import numpy as np
import pytest

import oracle
import synth


def _has_identical_reads(g):
    iv = np.stack([g.truth["start"], g.truth["end"]], axis=1)
    return len(np.unique(iv, axis=0)) != len(iv)


@pytest.mark.parametrize("seed,G,cov,extra", [(11, 300_000, 20, 0.0), (12, 1_000_000, 30, 0.0),
                                              (13, 1_000_000, 15, 0.02), (14, 600_000, 40, 0.01)])
def test_reduction_recovers_the_string_graph(seed, G, cov, extra):
    g = synth.simulate(G=G, cov=cov, mean_len=10_000, sd_len=3_000, err=0.0, extra_rate=extra,
                       seed=seed)
    if _has_identical_reads(g):
        pytest.skip("identical reads: the generator breaks that tie by its own index")
    r = synth.overlap_graph(g)
    assert r.m > 4 * g.m  # a real overlap graph, far from reduced
    contained, kept, s = oracle.reduce(r)
    assert np.array_equal(contained.astype(bool), g.truth["contained"])
    assert s.m == g.m and int(kept.sum()) == g.m
    for f in ("row_ptr", "col", "ovl", "strand"):
        assert np.array_equal(getattr(s, f), getattr(g, f)), f
    # and the path gives the same contigs on either graph
    a, b = oracle.run(s, P=8), oracle.run(g, P=8)
    assert np.array_equal(a["contigs"]["bases"], b["contigs"]["bases"])


def _reads(lens):
    rng = np.random.default_rng(0)
    return [rng.integers(0, 4, size=k).astype(np.uint8) for k in lens]


def test_contained_reads():
    # x covers all of y; of the equal reads p, q the smaller id stays
    g = synth.graph_from_edges(_reads([100, 50, 80, 80]),
                               [(0, 1, 50, 0, 0), (2, 3, 80, 0, 0), (0, 2, 30, 0, 0)])
    contained, kept, s = oracle.reduce(g)
    assert contained.tolist() == [0, 1, 0, 1]
    assert s.m == 2 and s.col.tolist() == [2, 0]  # only x - p is left


def _triangle(ov_ac, bits=((0, 0), (0, 0), (0, 0))):
    # a = [0, 100), b = [30, 130), c = [60, 160): overlaps 70, 70 and 40
    (sab, dab), (sbc, dbc), (sac, dac) = bits
    return synth.graph_from_edges(_reads([100, 100, 100]),
                                  [(0, 1, 70, sab, dab), (1, 2, 70, sbc, dbc),
                                   (0, 2, ov_ac, sac, dac)])


def test_transitive_edge_of_a_triangle():
    contained, kept, s = oracle.reduce(_triangle(40))
    assert not contained.any()
    assert s.m == 4 and s.col.tolist() == [1, 0, 2, 1]  # a-b and b-c stay, a-c goes
    # an overhang one base off is another path: kept, unless the fuzz allows it
    assert oracle.reduce(_triangle(41))[2].m == 6
    assert oracle.reduce(_triangle(41), fuzz=1)[2].m == 4


def test_walk_through_the_middle_read_must_be_valid():
    # b entered on one strand and left on the other: not a valid walk
    bad = oracle.reduce(_triangle(40, bits=((0, 0), (1, 1), (0, 1))))[2]
    assert bad.m == 6
    # the same triangle with consistent strands (all reads on their
    # reverse strand, walked the same way) is reduced
    good = oracle.reduce(_triangle(40, bits=((1, 1), (1, 1), (1, 1))))[2]
    assert good.m == 4


def test_ids_do_not_matter_and_reduction_is_idempotent():
    g = synth.simulate(G=400_000, cov=25, mean_len=8_000, sd_len=2_000, err=0.0,
                       extra_rate=0.02, seed=21)
    r = synth.overlap_graph(g)
    c, kept, s = oracle.reduce(r)
    assert oracle.validate(s)[0] == -1
    assert oracle.reduce(s)[2].m == s.m
    # relabel the reads: the reduced graph is relabelled the same way
    rng = np.random.default_rng(5)
    perm = rng.permutation(r.n)          # new id of old id i is perm[i]
    rows = np.repeat(np.arange(r.n), np.diff(r.row_ptr))
    pr = dataclasses.replace(r)
    src, dst = perm[rows], perm[r.col]
    order = np.lexsort((dst, src))
    pr.row_ptr = np.concatenate([[0], np.cumsum(np.bincount(src, minlength=r.n))]).astype(np.int32)
    pr.col = dst[order].astype(np.int32)
    pr.ovl = r.ovl[order]
    pr.strand = r.strand[order]
    inv = np.argsort(perm)
    pr.read_len = r.read_len[inv]
    pc, pk, ps = oracle.reduce(pr)
    assert np.array_equal(pc[perm], c)
    assert ps.m == s.m
    srows = np.repeat(np.arange(s.n), np.diff(s.row_ptr))
    want = sorted(zip(perm[srows].tolist(), perm[s.col].tolist()))
    prow = np.repeat(np.arange(ps.n), np.diff(ps.row_ptr))
    assert sorted(zip(prow.tolist(), ps.col.tolist())) == want


def test_a_hub_keeps_its_first_neighbour_only():
    # hub read 0 overlaps reads 1..k, each read i also overlaps read i + 1,
    # with overhangs making 0 -> i -> i+1 exactly as long as 0 -> i+1
    k = 40
    rng = np.random.default_rng(1)
    reads = [rng.integers(0, 4, size=100_000).astype(np.uint8)] + \
            [rng.integers(0, 4, size=10_000).astype(np.uint8) for _ in range(k)]
    edges = [(0, i, 10_000 - 5 * i, 0, 0) for i in range(1, k + 1)]
    edges += [(i, i + 1, 9_995, 0, 0) for i in range(1, k)]
    c, kept, s = oracle.reduce(synth.graph_from_edges(reads, edges))
    assert not c.any()
    assert s.row_ptr[1] == 1 and s.col[0] == 1
    assert s.m == 2 * k

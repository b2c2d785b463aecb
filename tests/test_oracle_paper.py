"""Oracle pinned to the worked examples the paper prints (tests/golden)."""
import numpy as np
import pytest

import oracle
import synth
from tests import brute


def _graph_from_golden(edges, n, read_len=20):
    reads = [np.zeros(read_len, np.uint8) for _ in range(n)]
    return synth.graph_from_edges(reads, [(a, b, 5, 0, 0) for a, b in edges])


def test_masking_example(golden):
    ex = golden["masking"]
    g = _graph_from_golden(ex["edges"], 8)
    assert oracle.validate(g) == (-1, 0)
    flags, counts = oracle.mask(g.n, g.row_ptr, g.col)
    assert sorted(np.nonzero(flags & 1)[0].tolist()) == ex["branch_vertices"]
    kept = set()
    for v in range(g.n):
        for j in range(2):
            if flags[v] & (2 << j):
                u = int(g.col[g.row_ptr[v] + j])
                kept.add((min(u, v), max(u, v)))
    assert sorted(kept) == sorted(tuple(e) for e in ex["kept_edges"])
    assert counts.tolist() == [1, 2 * len(ex["kept_edges"])]
    label = oracle.components(g.n, g.row_ptr, g.col, flags)
    for comp in ex["components"]:
        assert set(label[comp].tolist()) == {min(comp)}
    # the branch vertex is isolated in L and labels itself
    assert label[2] == 2


@pytest.mark.parametrize("P", [2, 3])
def test_lpt_example(golden, P):
    ex = golden["lpt"]
    g = _graph_from_golden(golden["masking"]["edges"], 8)
    r = oracle.run(g, P=P)
    parts = r["parts"]
    sizes = {str(l): int(s) for l, s in zip(parts["comp_label"], parts["comp_size"])}
    assert sizes == ex["sizes_by_label"]
    got = {str(l): int(b) for l, b in zip(parts["comp_label"], parts["comp_bin"])}
    assert got == ex["P%d" % P]["bin_by_label"]
    assert parts["bin_load"].tolist() == ex["P%d" % P]["loads"]


def _chain3(reads, ov, bits, ids=(0, 1, 2)):
    """Three reads joined ids[0]-ids[1]-ids[2] with entry bits for the walk
    direction reads[0] -> reads[1] -> reads[2]."""
    n = 3
    placed = [None] * n
    for r, i in zip(reads, ids):
        placed[i] = synth.encode(r)
    e = [(ids[0], ids[1], ov[0], bits[0][0], bits[0][1]),
         (ids[1], ids[2], ov[1], bits[1][0], bits[1][1])]
    return synth.graph_from_edges(placed, e)


def _contigs(g, P=1, min_reads=2):
    r = oracle.run(g, P=P, min_reads=min_reads)
    c = r["contigs"]
    return [synth.decode(oracle.contig_codes(c, k)) for k in range(len(c["len"]))], r


def test_fig3_concatenation(golden):
    ex = golden["concatenation"]
    g = _chain3(ex["reads"], ex["exact_overlaps"], [(0, 0), (0, 0)])
    assert oracle.validate(g) == (-1, 0)
    contigs, r = _contigs(g)
    assert contigs == [ex["contig"]]
    c = r["contigs"]
    assert int(c["len"][0]) == sum(len(s) for s in ex["reads"]) - sum(ex["exact_overlaps"])
    assert c["layout_vid"].tolist() == [0, 1, 2]
    assert c["layout_rev"].tolist() == [0, 0, 0]


def test_fig3_pre_post_printed_values(golden):
    """The paper's (pre, post) on l0 -> l1 is (1, 0): with an exact overlap of
    4 bases, pre is the last base of l0 before the overlap (inclusive
    indexing) and post the first overlapping base of l1."""
    ex = golden["concatenation"]
    l0, l1 = ex["reads"][0], ex["reads"][1]
    ov = ex["exact_overlaps"][0]
    pre, post = ex["pre_post"][0]
    assert len(l0) - ov - 1 == pre and post == 0
    assert l0[pre + 1:] == l1[post:post + ov]


def test_reverse_strand_example(golden):
    ex = golden["reverse_strand"]
    # l1 is stored reverse-complemented: it is entered reversed from l0 and
    # left reversed toward l2
    g = _chain3(ex["reads"], [4, 5], [(0, 1), (1, 0)])
    assert oracle.validate(g) == (-1, 0)
    contigs, r = _contigs(g)
    assert contigs == [ex["contig"]]
    assert r["contigs"]["layout_rev"].tolist() == [0, 1, 0]
    # the first overlapping base of l1 in its stored coordinates is |l1|-1
    assert ex["post_e0_by_definition"] == len(ex["reads"][1]) - 1
    # number the reads so that l2 is the smaller-id root: the walk starts there
    g2 = _chain3(ex["reads"], [4, 5], [(0, 1), (1, 0)], ids=(2, 1, 0))
    contigs2, r2 = _contigs(g2)
    assert contigs2 == [ex["contig_from_other_end"]]
    assert contigs2[0] == brute.revcomp(ex["contig"])
    assert r2["contigs"]["start"].tolist() == [0]


def test_reverse_complement_example(golden):
    ex = golden["reverse_complement"]
    # a read walked reversed contributes its reverse complement: a two-read
    # chain whose first read is left reversed starts with revcomp(l0)
    l0 = ex["seq"]
    rc = ex["revcomp"]
    l1 = rc[-3:] + "GG"
    g = synth.graph_from_edges([synth.encode(l0), synth.encode(l1)], [(0, 1, 3, 1, 0)])
    assert oracle.validate(g) == (-1, 0)
    contigs, _ = _contigs(g)
    assert contigs == [rc[:-3] + l1]
    assert contigs[0].startswith(rc)

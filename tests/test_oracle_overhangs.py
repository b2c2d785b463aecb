"""Explicit per-entry alignment coordinates (pre, post) of Section 4.4: the
oracle against the paper's x-drop example, against the overlap-length
reading, and against a direct transcription of the concatenation formula."""
import numpy as np
import pytest

import oracle
import synth
from tests import brute
from tests.test_oracle_paper import _chain3, _contigs


def _entry(g, u, v):
    for j in range(g.row_ptr[u], g.row_ptr[u + 1]):
        if g.col[j] == v:
            return j
    raise KeyError((u, v))


def _set(g, values):
    """values: {(u, v): (pre, post)} for every entry."""
    g.pre = np.zeros(g.m, np.uint32)
    g.post = np.zeros(g.m, np.uint32)
    for (u, v), (a, b) in values.items():
        j = _entry(g, u, v)
        g.pre[j], g.post[j] = a, b
    return g


def test_fig3_xdrop_example(golden):
    """Section 4.4: the alignment of l1 and l2 covers l1[5:7] and l2[2:4]
    only, so (pre, post) = (4, 2); with (1, 0) on l0 -> l1 the contig is the
    same as with exact overlaps."""
    ex = golden["concatenation"]
    g = _chain3(ex["reads"], ex["exact_overlaps"], [(0, 0), (0, 0)])
    (pa, qa), (pb, qb) = ex["pre_post"]
    # twin entries describe the same alignments walked the other way
    _set(g, {(0, 1): (pa, qa), (1, 2): (pb, qb), (1, 0): (4, 5), (2, 1): (5, 7)})
    assert oracle.validate(g) == (-1, 0)
    contigs, r = _contigs(g)
    assert contigs == [ex["contig"]]
    # pieces: l0[0:1] + l1[0:4] + l2[2:6]
    assert ex["contig"] == ex["reads"][0][:2] + ex["reads"][1][:5] + ex["reads"][2][2:]
    # pairing pre = 4 with post = 0 (ignoring the overhang) is wrong, as the
    # paper warns: l2's first two bases would be repeated
    _set(g, {(0, 1): (pa, qa), (1, 2): (pb, 0), (1, 0): (4, 5), (2, 1): (5, 7)})
    bad, _ = _contigs(g)
    assert bad == [ex["reads"][0][:2] + ex["reads"][1][:5] + ex["reads"][2]]
    assert bad != [ex["contig"]]


def test_reverse_strand_explicit(golden):
    """l1 stored reverse-complemented: post(e0) = 7 (reading: the printed 4 is
    not the first overlapping index of l1) and pre(e1) = 3 in l1's stored
    coordinates, walked downward."""
    ex = golden["reverse_strand"]
    g = _chain3(ex["reads"], [4, 5], [(0, 1), (1, 0)])
    _set(g, {(0, 1): (1, ex["post_e0_by_definition"]), (1, 2): (3, 2),
             (1, 0): (3, 5), (2, 1): (5, 0)})
    assert oracle.validate(g) == (-1, 0)
    contigs, _ = _contigs(g)
    assert contigs == [ex["contig"]]


def _random_graphs():
    rng = np.random.default_rng(31)
    gs = [synth.adversarial(rng) for _ in range(120)]
    gs.append(synth.config_graph(1))
    return gs


def test_exact_coordinates_match_the_overlap_reading():
    """pre/post derived from the overlaps reproduce the overlap-length path:
    the same walks everywhere and the same bases in every contig whose walk
    is valid.  (A same-end join, which Section 2 calls an invalid walk, reads
    pre from the entry's own strand bit here and from the walking orientation
    in the overlap reading; those contigs may differ.)"""
    n_sej = 0
    for i, g in enumerate(_random_graphs()):
        h = synth.with_alignment_ends(g, max_clip=0)
        for P, mr in ((3, 1), (8, 2)):
            a, b = oracle.run(g, P=P, min_reads=mr)["contigs"], oracle.run(h, P=P, min_reads=mr)["contigs"]
            for key in ("label", "start", "n_reads", "cflags", "layout_vid", "layout_rev"):
                assert np.array_equal(a[key], b[key]), (i, key)
            for k in range(len(a["len"])):
                if a["cflags"][k] & 2:
                    n_sej += 1
                    continue
                assert a["len"][k] == b["len"][k], (i, k)
                assert np.array_equal(oracle.contig_codes(a, k), oracle.contig_codes(b, k)), (i, k)
    assert n_sej > 0  # the corpus does exercise the excluded case


def test_consistent_clips_keep_error_free_contigs():
    """An alignment that starts late on both reads moves the join inside the
    overlap; with error-free reads the contig bases are unchanged."""
    g = synth.batch_graphs(only=[3])[0]
    h = synth.with_alignment_ends(g, np.random.default_rng(2), max_clip=3)
    assert np.any(h.pre != synth.with_alignment_ends(g, max_clip=0).pre)
    a, b = oracle.run(g, P=64), oracle.run(h, P=64)
    assert np.array_equal(a["contigs"]["len"], b["contigs"]["len"])
    assert np.array_equal(a["contigs"]["bases"], b["contigs"]["bases"])


def _random_pre_post(g, rng):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    h = synth.StringGraph(**{k: getattr(g, k) for k in ("n", "m", "row_ptr", "col", "ovl",
                                                       "strand", "read_len", "read_off", "seq")})
    h.pre = np.array([rng.integers(0, g.read_len[u]) for u in src], np.uint32)
    h.post = np.array([rng.integers(0, g.read_len[v]) for v in g.col], np.uint32)
    return h


def test_pieces_follow_the_concatenation_formula():
    """Brute force: walk each contig's layout and concatenate
    l[post(e_in) : pre(e_out)] directly (reverse complement when the read is
    walked reversed; empty when the range runs backwards)."""
    rng = np.random.default_rng(7)
    for i, g in enumerate(_random_graphs()[:100]):
        h = _random_pre_post(g, rng)
        assert oracle.validate(h) == (-1, 0)
        r = oracle.run(h, P=3, min_reads=1)
        c = r["contigs"]
        reads = [synth.decode(synth.unpack_read(h, v)) for v in range(h.n)]
        for k in range(len(c["len"])):
            lo, q = int(c["layout_off"][k]), int(c["n_reads"][k])
            vids = c["layout_vid"][lo:lo + q].tolist()
            revs = c["layout_rev"][lo:lo + q].tolist()
            want = ""
            for t, (v, o) in enumerate(zip(vids, revs)):
                L = len(reads[v])
                a = (L - 1 if o else 0) if t == 0 else int(h.post[_entry(h, vids[t - 1], v)])
                b = (0 if o else L - 1) if t == q - 1 else int(h.pre[_entry(h, v, vids[t + 1])])
                if not o:
                    want += reads[v][a:b + 1] if b >= a else ""
                else:
                    want += brute.revcomp(reads[v][b:a + 1]) if a >= b else ""
            got = synth.decode(oracle.contig_codes(c, k))
            assert got == want, (i, k)


def test_coordinates_outside_their_reads_are_rejected():
    g = synth.config_graph(1)
    h = synth.with_alignment_ends(g, max_clip=0)
    assert oracle.validate(h) == (-1, 0)
    src = np.repeat(np.arange(h.n), np.diff(h.row_ptr))
    e = int(np.nonzero(h.pre >= 0)[0][5])
    bad = synth.with_alignment_ends(g, max_clip=0)
    bad.pre = h.pre.copy()
    bad.pre[e] = h.read_len[src[e]]
    assert oracle.validate(bad) == (e, 12)
    bad = synth.with_alignment_ends(g, max_clip=0)
    bad.post = h.post.copy()
    bad.post[e] = h.read_len[h.col[e]]
    assert oracle.validate(bad) == (e, 13)

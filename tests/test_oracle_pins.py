"""Oracle pinned to brute force, closed forms and invariants.

Each check uses a method other than the oracle's own: breadth-first search
for components, exhaustive path enumeration for chain layouts, string
operations for contigs, exhaustive search for the LPT optimum, Graham's
bounds and tight family, and the true genome for error-free chains.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import brute


def _adversarial_corpus(count, seed=7):
    rng = np.random.default_rng(seed)
    return [synth.adversarial(rng) for _ in range(count)]


CORPUS = _adversarial_corpus(400)


def _check_graph(g, P, min_reads):
    assert oracle.validate(g) == (-1, 0)
    r = oracle.run(g, P=P, min_reads=min_reads)
    flags, label, parts, local, c = r["flags"], r["label"], r["parts"], r["local"], r["contigs"]
    ent = brute.entries(g)

    # mask: degree from column counts, branch at >= 3, kept iff no branch end
    deg, branch, kept = brute.bf_mask(g)
    assert sorted(np.nonzero(flags & 1)[0].tolist()) == sorted(branch)
    got_kept = set()
    for v in range(g.n):
        for j in range(2):
            if flags[v] & (2 << j):
                got_kept.add((v, int(g.col[g.row_ptr[v] + j])))
    assert got_kept == kept
    assert r["counts"].tolist() == [len(branch), len(kept)]
    degL = np.zeros(g.n, np.int64)
    for (u, _v) in kept:
        degL[u] += 1
    assert degL.max(initial=0) <= 2

    # components: BFS on L, smallest id
    bl, adj = brute.bf_components(g.n, kept)
    assert label.tolist() == bl.tolist()

    # table: sizes sum to n over all labels; eligible ones in label order
    sizes = np.bincount(bl, minlength=g.n)
    assert sizes.sum() == g.n
    mr = max(min_reads, 1)
    want = [r_ for r_ in range(g.n) if sizes[r_] >= mr and r_ not in branch and bl[r_] == r_]
    assert parts["comp_label"].tolist() == want
    for k, lab in enumerate(want):
        verts = [v for v in range(g.n) if bl[v] == lab]
        e = sum(degL[v] for v in verts) // 2
        q = len(verts)
        kind = parts["comp_kind"][k]
        assert parts["comp_size"][k] == q
        assert kind == (oracle.SINGLE if q == 1 else oracle.PATH if e == q - 1 else oracle.CYCLE)
        assert e in (q - 1, q)
        assert parts["label_comp"][lab] == k
    assert (parts["label_comp"] >= 0).sum() == len(want)

    # LPT: loads equal the sizes placed; makespan within Graham's bound
    nc = len(want)
    loads = np.zeros(P, np.int64)
    for k in range(nc):
        loads[parts["comp_bin"][k]] += parts["comp_size"][k]
    assert loads.tolist() == parts["bin_load"].astype(np.int64).tolist()
    if nc:
        lb = max(int(parts["comp_size"].max()), math.ceil(int(parts["comp_size"].sum()) / P))
        assert loads.max() >= lb
        assert 3 * P * loads.max() <= (4 * P - 1) * lb * 2    # loose: OPT <= 2*lb for LPT
        # the first min(P, nc) components in LPT order take bins 0, 1, 2, ...
        order = sorted(range(nc), key=lambda k: (-parts["comp_size"][k], parts["comp_label"][k]))
        for i, k in enumerate(order[:P]):
            assert parts["comp_bin"][k] == i

    # (bin, label) order and read offsets
    ranks = parts["comp_rank"]
    assert sorted(ranks.tolist()) == list(range(nc))
    by_rank = sorted(range(nc), key=lambda k: (parts["comp_bin"][k], parts["comp_label"][k]))
    assert [int(ranks[k]) for k in by_rank] == list(range(nc))
    acc = 0
    for k in by_rank:
        assert parts["comp_start"][k] == acc
        acc += int(parts["comp_size"][k])

    # induce: perm is the eligible vertices in (bin, label, id) order; the
    # local CSR holds exactly the kept entries, renumbered
    elig = [v for v in range(g.n) if parts["label_comp"][bl[v]] >= 0]
    key = lambda v: (parts["comp_bin"][parts["label_comp"][bl[v]]], bl[v], v)
    assert local["perm"].tolist() == sorted(elig, key=key)
    perm = local["perm"]
    assert local["n_e"] == len(elig)
    for i in range(local["n_e"]):
        v = int(perm[i])
        a, b = local["loc_row_ptr"][i], local["loc_row_ptr"][i + 1]
        assert b - a == degL[v]
        for t in range(a, b):
            e = int(local["loc_eid"][t])
            assert g.row_ptr[v] <= e < g.row_ptr[v + 1]
            assert int(g.col[e]) == int(perm[local["loc_col"][t]])
    bv = local["bin_vptr"]
    for b in range(P):
        assert bv[b + 1] - bv[b] == loads[b]

    # assemble: layout is a Hamiltonian path of the component (brute-force
    # enumeration), started at the smaller root, bytes by string operations
    seen = []
    for k in range(nc):
        lo = int(c["layout_off"][k])
        q = int(c["n_reads"][k])
        walk = c["layout_vid"][lo:lo + q].tolist()
        seen += walk
        verts = sorted(v for v in range(g.n) if bl[v] == c["label"][k])
        assert sorted(walk) == verts
        kind = parts["comp_kind"][parts["label_comp"][c["label"][k]]]
        if q > 1:
            hp = brute.hamiltonian_paths(verts, adj)
            assert walk in hp
            if kind == oracle.PATH:
                ends = [v for v in verts if degL[v] == 1]
                assert walk[0] == min(ends)
            else:
                assert walk[0] == verts[0]
                nb = sorted(y for y in adj[verts[0]])
                assert walk[1] == nb[0]
        s, orient, sej = brute.contig_from_walk(g, walk, ent)
        assert synth.decode(oracle.contig_codes(c, k)) == s
        assert c["layout_rev"][lo:lo + q].tolist() == orient
        assert int(c["len"][k]) == sum(int(g.read_len[v]) for v in walk) - sum(
            ent[(x, y)][0] for x, y in zip(walk[:-1], walk[1:]))
        assert bool(c["cflags"][k] & oracle.SAME_END_JOIN) == sej
        assert bool(c["cflags"][k] & oracle.CIRCULAR) == (kind == oracle.CYCLE)
        assert bool(c["cflags"][k] & oracle.SINGLE_READ) == (q == 1)
        assert c["base_off"][k] % 16 == 0
    assert sorted(seen) == sorted(elig)
    # padding bits past each contig's end are zero
    for k in range(nc):
        L = int(c["len"][k])
        if L % 16:
            w = int(c["bases"][(int(c["base_off"][k]) + L) // 16])
            assert w >> (2 * (L % 16)) == 0
    return r


@pytest.mark.parametrize("i", range(len(CORPUS)))
def test_adversarial(i):
    g = CORPUS[i]
    rng = np.random.default_rng(1000 + i)
    P = int(rng.integers(1, 6))
    min_reads = int(rng.integers(1, 3))
    _check_graph(g, P, min_reads)


def test_corpus_covers_the_hard_cases():
    """The corpus really contains cycles, same-end joins, singletons,
    branch vertices and more bins than components."""
    seen = dict(cycle=0, sej=0, single=0, branch=0, idle_bins=0)
    for i, g in enumerate(CORPUS):
        r = oracle.run(g, P=4, min_reads=1)
        cf = r["contigs"]["cflags"]
        seen["cycle"] += int((cf & oracle.CIRCULAR).astype(bool).sum())
        seen["sej"] += int((cf & oracle.SAME_END_JOIN).astype(bool).sum())
        seen["single"] += int((cf & oracle.SINGLE_READ).astype(bool).sum())
        seen["branch"] += int(r["counts"][0])
        seen["idle_bins"] += int((r["parts"]["bin_load"] == 0).sum())
    assert all(v > 10 for v in seen.values()), seen


@pytest.mark.parametrize("P", [2, 3, 4])
def test_lpt_graham_tight_family(P):
    sizes = brute.graham_family(P)
    labels = list(range(len(sizes)))
    comp_bin, loads = oracle.lpt(np.array(sizes, np.int32), np.array(labels, np.int32), P)
    assert int(loads.max()) == 4 * P - 1
    assert brute.lpt_opt(sizes, P) == 3 * P


def test_lpt_against_exhaustive_optimum():
    rng = np.random.default_rng(3)
    for _ in range(150):
        P = int(rng.integers(1, 5))
        nc = int(rng.integers(0, 8))
        sizes = rng.integers(1, 20, size=nc).astype(np.int32)
        labels = np.sort(rng.choice(1000, size=nc, replace=False)).astype(np.int32)
        comp_bin, loads = oracle.lpt(sizes, labels, P)
        opt = brute.lpt_opt(sizes.tolist(), P)
        mk = int(loads.max()) if P else 0
        assert mk * 3 * P <= (4 * P - 1) * opt
        assert mk >= max(int(sizes.max(initial=0)), math.ceil(int(sizes.sum()) / P))
        # the greedy rule itself, replayed from the definition
        ld = [0] * P
        for k in sorted(range(nc), key=lambda k: (-sizes[k], labels[k])):
            b = min(range(P), key=lambda j: (ld[j], j))
            assert comp_bin[k] == b
            ld[b] += int(sizes[k])


def _error_free_sim(seed, G=300_000, extra=0.02):
    return synth.simulate(G=G, cov=15, mean_len=5_000, sd_len=1_500, err=0.0,
                          extra_rate=extra, seed=seed)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_closed_form_error_free_chains(seed):
    """A chain of error-free reads joined only by true overlaps spells the
    genome between its first read's start and its last read's end, on one
    strand or the other."""
    g = _error_free_sim(seed)
    G = g.truth["genome"]
    gstr = synth.decode(G)
    extra = {tuple(sorted(e)) for e in g.truth["extra_edges"].tolist()}
    r = oracle.run(g, P=8, min_reads=2)
    c = r["contigs"]
    checked = 0
    for k in range(len(c["len"])):
        lo, q = int(c["layout_off"][k]), int(c["n_reads"][k])
        walk = c["layout_vid"][lo:lo + q].tolist()
        if any(tuple(sorted((x, y))) in extra for x, y in zip(walk[:-1], walk[1:])):
            continue
        a = g.truth["start"][walk]
        b = g.truth["end"][walk]
        seg = gstr[int(a.min()):int(b.max())]
        got = synth.decode(oracle.contig_codes(c, k))
        forward = a[-1] > a[0]
        assert got == (seg if forward else brute.revcomp(seg))
        # the walk orientation agrees with the strand each read was drawn from
        assert (c["layout_rev"][lo:lo + q] == (g.truth["rc"][walk] ^ (0 if forward else 1))).all()
        checked += 1
    assert checked > 5


@pytest.mark.parametrize("seed", [21, 22])
def test_every_non_branch_read_in_one_contig(seed):
    g = _error_free_sim(seed)
    r = oracle.run(g, P=16, min_reads=1)
    non_branch = np.nonzero((r["flags"] & 1) == 0)[0]
    c = r["contigs"]
    assert np.array_equal(np.sort(c["layout_vid"]), non_branch)
    lens = g.read_len.astype(np.int64)
    ent = brute.entries(g)
    for k in range(len(c["len"])):
        lo, q = int(c["layout_off"][k]), int(c["n_reads"][k])
        w = c["layout_vid"][lo:lo + q].tolist()
        assert int(c["len"][k]) == lens[w].sum() - sum(ent[(x, y)][0] for x, y in zip(w[:-1], w[1:]))


def _relabel(g, newid):
    """Same graph with vertex v renamed newid[v] (reads move with it)."""
    n = g.n
    inv = np.empty(n, np.int64)
    inv[newid] = np.arange(n)
    reads = [synth.unpack_read(g, int(inv[i])) for i in range(n)]
    edges = []
    for u in range(n):
        for j in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            v = int(g.col[j])
            if u < v:
                b = int(g.strand[j])
                edges.append((int(newid[u]), int(newid[v]), int(g.ovl[j]), b & 1, (b >> 1) & 1))
    return synth.graph_from_edges(reads, edges)


def test_reversal_gives_reverse_complement():
    """Numbering the reads in reverse swaps which root starts each path; for
    error-free reads the contig then reads as the reverse complement."""
    g = _error_free_sim(31, G=150_000)
    r1 = oracle.run(g, P=4, min_reads=2)
    newid = (g.n - 1 - np.arange(g.n)).astype(np.int64)
    g2 = _relabel(g, newid)
    r2 = oracle.run(g2, P=4, min_reads=2)
    c1, c2 = r1["contigs"], r2["contigs"]
    by_set = {}
    for k in range(len(c2["len"])):
        lo, q = int(c2["layout_off"][k]), int(c2["n_reads"][k])
        by_set[frozenset(c2["layout_vid"][lo:lo + q].tolist())] = k
    swapped = 0
    for k in range(len(c1["len"])):
        lo, q = int(c1["layout_off"][k]), int(c1["n_reads"][k])
        w = c1["layout_vid"][lo:lo + q]
        k2 = by_set[frozenset(newid[w].tolist())]
        s1 = synth.decode(oracle.contig_codes(c1, k))
        s2 = synth.decode(oracle.contig_codes(c2, k2))
        cyc = bool(c1["cflags"][k] & oracle.CIRCULAR)
        if not cyc and newid[w[0]] != c2["start"][k2]:
            assert s2 == brute.revcomp(s1)
            swapped += 1
        elif not cyc:
            assert s2 == s1
    assert swapped > 0


def test_config1_invariants():
    g = synth.config_graph(1)
    assert oracle.validate(g) == (-1, 0)
    r = oracle.run(g, P=8, min_reads=2)
    c = r["contigs"]
    assert len(c["len"]) == r["parts"]["n_comp"] > 0
    assert int(c["len"].sum()) > 0.8 * g.meta["G"]
    assert (np.diff(c["base_off"].astype(np.int64)) ==
            16 * ((c["len"][:-1].astype(np.int64) + 15) // 16)).all()


NEGATIVE = {
    "asymmetric": 5, "bad_twin_bits": 7, "ovl_too_long": 8, "self_loop": 3, "duplicate": 4,
    "twin_ovl": 6, "misaligned_read": 10, "pre_outside_read": 12, "post_outside_read": 13,
}


def break_graph(g, case):
    """The negative case `case` planted into a valid 4-read graph."""
    if case == "asymmetric":
        g.col = g.col.copy()
        g.col[0] = 3          # 0->3 has no twin
    elif case == "bad_twin_bits":
        g.strand = g.strand.copy()
        g.strand[0] ^= 1
    elif case == "ovl_too_long":
        g.ovl = g.ovl.copy()
        g.ovl[:] = 10
    elif case == "self_loop":
        g.col = g.col.copy()
        g.col[0] = 0
    elif case == "duplicate":
        g.col = g.col.copy()
        g.col[2] = g.col[1]
    elif case == "twin_ovl":
        g.ovl = g.ovl.copy()
        g.ovl[0] = 4
    elif case == "misaligned_read":
        g.read_off = g.read_off.copy()
        g.read_off[1] += 1
    elif case == "pre_outside_read":
        g = synth.with_alignment_ends(g)
        g.pre[0] = g.read_len[0]   # entry 0 is (0, 1): pre indexes read 0
    elif case == "post_outside_read":
        g = synth.with_alignment_ends(g)
        g.post[0] = g.read_len[1]  # post indexes read 1
    return g


@pytest.mark.parametrize("case", sorted(NEGATIVE))
def test_validate_rejects(case):
    reads = [np.zeros(10, np.uint8) for _ in range(4)]
    g = synth.graph_from_edges(reads, [(0, 1, 3, 0, 0), (1, 2, 3, 1, 0)])
    assert oracle.validate(g) == (-1, 0)
    g = break_graph(g, case)
    bad, why = oracle.validate(g)
    assert bad != -1 and why == NEGATIVE[case]

"""Seeded synthetic string graphs shaped like long-read assembly workloads.

Input synthesis only.  This module simulates a genome, samples long reads from
it, drops contained reads, links consecutive surviving reads into the exact
transitively reduced string graph (from their true genome positions), adds
random extra overlap edges that create branch vertices, shuffles vertex ids and
packs the reads 2 bits per base.  It holds none of the contig-generation
method's arithmetic (no degrees, components, partitions, walks or contigs):
both the oracle tests and the GPU path read its output, and neither shares any
other code with it.

Data layout of a graph (all numpy, host memory):

* ``row_ptr`` int32[n+1], ``col`` int32[m]: symmetric CSR, columns sorted
  within each row, no self loops, no duplicates.
* ``ovl`` uint32[m]: overlap length of the entry, equal in both directions,
  ``1 <= ovl < min(read_len[u], read_len[v])``.
* ``strand`` uint8[m]: bit0 ``s`` = u is reverse-complemented when the walk
  leaves u along this entry; bit1 ``d`` = v is reverse-complemented when the
  walk enters v along it.  The twin entry (v, u) carries (not d, not s).
* ``read_len`` uint32[n], ``read_off`` uint64[n] (multiple of 16), ``seq``
  uint32 words: base i of the store at bits 2*(i % 16) of word i // 16,
  A=0 C=1 G=2 T=3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 20220704
MIN_OVERLAP = 1000
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def build_helper(force: bool = False) -> str:
    """Compile the bulk read-extraction helper next to this file."""
    so = os.path.join(_HERE, "libsynth.so")
    src = os.path.join(_HERE, "_synth.c")
    if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
        tmp = so + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, so)
    return so


def _lib():
    global _LIB
    if _LIB is None:
        lib = ctypes.CDLL(build_helper())
        p = ctypes.c_void_p
        lib.synth_extract_reads.argtypes = [p, ctypes.c_int64, p, p, p, p, p, ctypes.c_int64]
        lib.synth_extract_reads.restype = None
        _LIB = lib
    return _LIB


@dataclass
class StringGraph:
    n: int
    m: int
    row_ptr: np.ndarray
    col: np.ndarray
    ovl: np.ndarray
    strand: np.ndarray
    read_len: np.ndarray
    read_off: np.ndarray
    seq: np.ndarray
    truth: dict = field(default_factory=dict)
    meta: dict = field(default_factory=dict)
    pre: np.ndarray = None     # optional alignment coordinates per entry (uint32[m])
    post: np.ndarray = None

    @property
    def seq_words(self) -> int:
        return int(self.seq.shape[0])

    def nbytes(self) -> int:
        return sum(a.nbytes for a in (self.row_ptr, self.col, self.ovl, self.strand,
                                      self.read_len, self.read_off, self.seq))


# ----------------------------------------------------------------------------
# Low-level builders (also used by hand-written test graphs)
# ----------------------------------------------------------------------------

def pack_reads(reads):
    """Pack a list of uint8 base-code arrays into the 2-bit store.

    Returns (read_len uint32, read_off uint64, seq uint32)."""
    lens = np.array([len(r) for r in reads], dtype=np.int64)
    words = (lens + 15) // 16
    offw = np.zeros(len(reads) + 1, dtype=np.int64)
    np.cumsum(words, out=offw[1:])
    seq = np.zeros(max(int(offw[-1]), 1), dtype=np.uint32)
    for i, r in enumerate(reads):
        r = np.asarray(r, dtype=np.uint32)
        pad = np.zeros(words[i] * 16, dtype=np.uint32)
        pad[: len(r)] = r & 3
        w = (pad.reshape(-1, 16) << (2 * np.arange(16, dtype=np.uint32))).sum(axis=1, dtype=np.uint64)
        seq[offw[i]: offw[i + 1]] = w.astype(np.uint32)
    return lens.astype(np.uint32), (offw[:-1] * 16).astype(np.uint64), seq


def unpack_read(g: StringGraph, v: int) -> np.ndarray:
    """Base codes of read v as stored (test helper)."""
    L = int(g.read_len[v])
    o = int(g.read_off[v])
    idx = o + np.arange(L, dtype=np.int64)
    return ((g.seq[idx >> 4] >> (2 * (idx & 15)).astype(np.uint32)) & 3).astype(np.uint8)


def csr_from_edges(n, u, v, ovl, s, d):
    """Symmetric CSR from undirected edges (u, v) with entry bits for u->v.

    The twin entry v->u gets (not d, not s) and the same overlap length."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    ovl = np.asarray(ovl, dtype=np.int64)
    s = np.asarray(s, dtype=np.int64) & 1
    d = np.asarray(d, dtype=np.int64) & 1
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    ov = np.concatenate([ovl, ovl])
    bits = np.concatenate([s | (d << 1), (1 - d) | ((1 - s) << 1)])
    order = np.lexsort((dst, src))
    src, dst, ov, bits = src[order], dst[order], ov[order], bits[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=row_ptr[1:])
    return (row_ptr.astype(np.int32), dst.astype(np.int32), ov.astype(np.uint32),
            bits.astype(np.uint8))


def graph_from_edges(reads, edges, meta=None):
    """Build a StringGraph from base-code reads and (u, v, ovl, s, d) tuples."""
    n = len(reads)
    read_len, read_off, seq = pack_reads(reads)
    if edges:
        e = np.array(edges, dtype=np.int64).reshape(-1, 5)
        row_ptr, col, ovl, strand = csr_from_edges(n, e[:, 0], e[:, 1], e[:, 2], e[:, 3], e[:, 4])
    else:
        row_ptr = np.zeros(n + 1, dtype=np.int32)
        col = np.zeros(0, dtype=np.int32)
        ovl = np.zeros(0, dtype=np.uint32)
        strand = np.zeros(0, dtype=np.uint8)
    return StringGraph(n=n, m=int(col.shape[0]), row_ptr=row_ptr, col=col, ovl=ovl,
                       strand=strand, read_len=read_len, read_off=read_off, seq=seq,
                       meta=dict(meta or {}))


def encode(s: str) -> np.ndarray:
    table = {"A": 0, "C": 1, "G": 2, "T": 3}
    return np.array([table[c] for c in s], dtype=np.uint8)


def decode(codes) -> str:
    return "".join("ACGT"[int(c)] for c in codes)


# ----------------------------------------------------------------------------
# Genome and read simulation
# ----------------------------------------------------------------------------

def _place_nonoverlapping(rng, G, lengths):
    """Uniform non-overlapping placement of intervals of the given lengths."""
    lengths = np.asarray(lengths, dtype=np.int64)
    free = G - int(lengths.sum())
    if free < 0:
        raise ValueError("repeat copies do not fit in the genome")
    order = rng.permutation(len(lengths))
    cuts = np.sort(rng.integers(0, free + 1, size=len(lengths)))
    starts = np.empty(len(lengths), dtype=np.int64)
    starts[order] = cuts + np.concatenate([[0], np.cumsum(lengths[order])[:-1]])
    return starts


def make_genome(rng, G, repeats=None):
    """iid uniform ACGT genome with optional repeat families overwritten in.

    repeats: None, ("fixed", families, copies, unit_len) or
             ("fraction", frac, unit_lo, unit_hi, copies_lo, copies_hi)."""
    genome = rng.integers(0, 4, size=G, dtype=np.uint8)
    info = {"families": 0, "copies": 0, "repeat_bases": 0}
    if repeats is None:
        return genome, info
    units, counts = [], []
    if repeats[0] == "fixed":
        _, fam, copies, unit_len = repeats
        for _ in range(fam):
            units.append(rng.integers(0, 4, size=unit_len, dtype=np.uint8))
            counts.append(copies)
    else:
        _, frac, ulo, uhi, clo, chi = repeats
        target = int(frac * G)
        total = 0
        while total < target:
            L = int(rng.integers(ulo, uhi + 1))
            c = int(rng.integers(clo, chi + 1))
            units.append(rng.integers(0, 4, size=L, dtype=np.uint8))
            counts.append(c)
            total += L * c
    lengths = np.concatenate([[len(u)] * c for u, c in zip(units, counts)]).astype(np.int64)
    starts = _place_nonoverlapping(rng, G, lengths)
    k = 0
    for u, c in zip(units, counts):
        for _ in range(c):
            genome[starts[k]: starts[k] + len(u)] = u
            k += 1
    info = {"families": len(units), "copies": int(sum(counts)), "repeat_bases": int(lengths.sum())}
    return genome, info


def lognormal_lengths(rng, n, mean, sd, lo, hi):
    s2 = np.log1p((sd / mean) ** 2)
    mu = np.log(mean) - s2 / 2
    x = rng.lognormal(mu, np.sqrt(s2), size=n)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def simulate(G, cov, mean_len, sd_len, err, extra_rate, seed, repeats=None, P=64,
             name="custom"):
    """One string graph from a simulated genome (see the module docstring)."""
    ss = np.random.SeedSequence(seed)
    r_genome, r_reads, r_err, r_extra, r_ids = [np.random.default_rng(s) for s in ss.spawn(5)]
    genome, rep_info = make_genome(r_genome, int(G), repeats)
    G = int(G)
    N = int(round(G * cov / mean_len))
    lens = lognormal_lengths(r_reads, N, mean_len, sd_len, 500, G)
    a = r_reads.integers(0, G - lens + 1)
    b = a + lens
    rc = (r_reads.random(N) < 0.5).astype(np.uint8)

    # containment: sort by (start asc, end desc, index asc); a read is
    # contained when an earlier read in that order reaches at least its end
    order = np.lexsort((np.arange(N), -b, a))
    bmax = np.maximum.accumulate(b[order])
    prev = np.concatenate([[-1], bmax[:-1]])
    contained = np.zeros(N, dtype=bool)
    contained[order] = prev >= b[order]

    # exact reduced graph: consecutive non-contained reads overlapping >= MIN_OVERLAP
    keep = order[~contained[order]]            # non-contained reads by start
    ov = b[keep[:-1]] - a[keep[1:]]
    link = ov >= MIN_OVERLAP
    tu, tv, tov = keep[:-1][link], keep[1:][link], ov[link]
    ts, td = rc[tu].astype(np.int64), rc[tv].astype(np.int64)

    # extra (branch) edges between non-adjacent non-contained reads
    n_extra = int(round(extra_rate * len(tu)))
    adjacent = set(zip(np.minimum(tu, tv).tolist(), np.maximum(tu, tv).tolist()))
    eu, ev, eov, es, ed = [], [], [], [], []
    attempts = 0
    while len(eu) < n_extra and len(keep) >= 2 and attempts < 50 * n_extra + 100:
        attempts += 1
        x, y = (int(t) for t in r_extra.choice(keep, size=2, replace=False))
        key = (min(x, y), max(x, y))
        if key in adjacent:
            continue
        hi = int(min(lens[x], lens[y])) - 1
        if hi < MIN_OVERLAP:
            continue
        adjacent.add(key)
        eu.append(x)
        ev.append(y)
        eov.append(int(r_extra.integers(MIN_OVERLAP, hi + 1)))
        es.append(int(r_extra.integers(0, 2)))
        ed.append(int(r_extra.integers(0, 2)))

    # shuffle vertex ids so that id order is file order, not genome order
    ids = r_ids.permutation(N)
    u = np.concatenate([ids[tu], ids[np.array(eu, dtype=np.int64)]])
    v = np.concatenate([ids[tv], ids[np.array(ev, dtype=np.int64)]])
    o = np.concatenate([tov, np.array(eov, dtype=np.int64)])
    s = np.concatenate([ts, np.array(es, dtype=np.int64)])
    d = np.concatenate([td, np.array(ed, dtype=np.int64)])
    row_ptr, col, ovl, strand = csr_from_edges(N, u, v, o, s, d)

    # reads in id order at 16-base-aligned offsets
    inv = np.empty(N, dtype=np.int64)
    inv[ids] = np.arange(N)
    len_id = lens[inv]
    words = (len_id + 15) // 16
    offw = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(words, out=offw[1:])
    seq = np.zeros(max(int(offw[-1]), 1), dtype=np.uint32)
    st = np.ascontiguousarray(a[inv], dtype=np.int64)
    ln = np.ascontiguousarray(len_id, dtype=np.int64)
    rcid = np.ascontiguousarray(rc[inv], dtype=np.uint8)
    off = np.ascontiguousarray(offw[:-1] * 16, dtype=np.int64)
    _lib().synth_extract_reads(genome.ctypes.data, N, st.ctypes.data, ln.ctypes.data,
                               rcid.ctypes.data, off.ctypes.data, seq.ctypes.data, seq.shape[0])
    if err > 0:
        _substitute(r_err, seq, off, ln, err)

    truth = {
        "start": a[inv], "end": b[inv], "rc": rcid, "contained": contained[inv],
        "extra_edges": np.stack([ids[np.array(eu, dtype=np.int64)],
                                 ids[np.array(ev, dtype=np.int64)]], axis=1)
        if eu else np.zeros((0, 2), dtype=np.int64),
        "genome_len": G,
    }
    meta = {"name": name, "G": G, "cov": cov, "mean_len": mean_len, "sd_len": sd_len,
            "err": err, "extra_rate": extra_rate, "seed": int(seed), "P": int(P),
            "non_contained": int(len(keep)), "true_edges": int(len(tu)),
            "extra_edges": int(len(eu)), **rep_info}
    g = StringGraph(n=N, m=int(col.shape[0]), row_ptr=row_ptr, col=col, ovl=ovl, strand=strand,
                    read_len=len_id.astype(np.uint32), read_off=off.astype(np.uint64), seq=seq,
                    truth=truth, meta=meta)
    g.truth["genome"] = genome if G <= 4_000_000 else None
    return g


def overlap_graph(g: StringGraph, min_overlap: int = MIN_OVERLAP) -> StringGraph:
    """The overlap graph g was reduced from (the input of Algorithm 1's
    pruning and transitive reduction): every pair of reads whose true
    intervals overlap by at least min_overlap bases, contained reads
    included, plus g's extra edges with g's values (an extra edge replaces a
    true overlap of the same pair).  A true pair's entry from the read that
    comes first in (start asc, end desc, id asc) order carries (its
    orientation, the other's), as g's edges do.  Same reads and ids as g."""
    import dataclasses
    n = g.n
    a = np.asarray(g.truth["start"], dtype=np.int64)
    b = np.asarray(g.truth["end"], dtype=np.int64)
    rc = np.asarray(g.truth["rc"], dtype=np.int64)
    order = np.lexsort((np.arange(n), -b, a))
    A, Bv = a[order], b[order]
    us, vs, ovs = [], [], []
    k = 1
    while k < n:
        i = np.arange(n - k)
        j = i + k
        cand = A[j] + min_overlap <= Bv[i]   # starts are sorted: none further once this fails
        if not cand.any():
            break
        ov = np.minimum(Bv[i], Bv[j]) - A[j]
        ok = cand & (ov >= min_overlap)
        us.append(order[i[ok]])
        vs.append(order[j[ok]])
        ovs.append(ov[ok])
        k += 1
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    o = np.concatenate(ovs) if ovs else np.zeros(0, np.int64)
    s_, d_ = rc[u], rc[v]
    extra = np.asarray(g.truth.get("extra_edges", np.zeros((0, 2))), dtype=np.int64).reshape(-1, 2)
    if len(extra):
        key = lambda x, y: np.minimum(x, y) * n + np.maximum(x, y)
        drop = np.isin(key(u, v), key(extra[:, 0], extra[:, 1]))
        u, v, o, s_, d_ = u[~drop], v[~drop], o[~drop], s_[~drop], d_[~drop]
        eu, ev, eo, es, ed = [], [], [], [], []
        for x, y in extra.tolist():
            lo, hi = int(g.row_ptr[x]), int(g.row_ptr[x + 1])
            jj = lo + int(np.searchsorted(g.col[lo:hi], y))
            eu.append(x)
            ev.append(y)
            eo.append(int(g.ovl[jj]))
            es.append(int(g.strand[jj]) & 1)
            ed.append((int(g.strand[jj]) >> 1) & 1)
        u = np.concatenate([u, eu])
        v = np.concatenate([v, ev])
        o = np.concatenate([o, eo])
        s_ = np.concatenate([s_, es])
        d_ = np.concatenate([d_, ed])
    row_ptr, col, ovl, strand = csr_from_edges(n, u, v, o, s_, d_)
    meta = dict(g.meta, overlap_graph=True, min_overlap=int(min_overlap))
    return dataclasses.replace(g, m=int(col.shape[0]), row_ptr=row_ptr, col=col, ovl=ovl,
                               strand=strand, meta=meta, pre=None, post=None)


def _substitute(rng, seq, off, ln, err):
    """Uniform substitution errors in the packed store, in place."""
    total = int(ln.sum())
    k = rng.binomial(total, err)
    pos = np.sort(rng.choice(total, size=k, replace=False)) if k else np.zeros(0, np.int64)
    cum = np.concatenate([[0], np.cumsum(ln)])
    r = np.searchsorted(cum, pos, side="right") - 1
    gi = off[r] + (pos - cum[r])
    delta = rng.integers(1, 4, size=k).astype(np.uint32)      # new = old + delta (mod 4)
    w = gi >> 4
    sh = (2 * (gi & 15)).astype(np.uint32)
    old = (seq[w] >> sh) & 3
    new = (old + delta) & 3
    np.bitwise_xor.at(seq, w, ((old ^ new) << sh).astype(np.uint32))


# ----------------------------------------------------------------------------
# The five workload configurations
# ----------------------------------------------------------------------------

CONFIGS = {
    1: dict(G=1_000_000, cov=10, mean_len=10_000, sd_len=3_000, err=0.05, extra_rate=0.01,
            repeats=None, P=8, name="plain-tiny-1Mbp"),
    2: dict(G=50_000_000, cov=30, mean_len=12_000, sd_len=4_000, err=0.0, extra_rate=0.02,
            repeats=("fixed", 10, 20, 8_000), P=64, name="plain-50Mbp"),
    3: dict(G=1_000_000_000, cov=20, mean_len=15_000, sd_len=5_000, err=0.0, extra_rate=0.01,
            repeats=("fraction", 0.05, 5_000, 15_000, 2, 20), P=1024, name="large-1Gbp"),
}


def config_graph(cfg: int, seed_offset: int = 0) -> StringGraph:
    """Single-graph configurations 1-3."""
    c = dict(CONFIGS[cfg])
    return simulate(seed=SEED_BASE + cfg + 1000 * seed_offset, **c)


def batch_params(n_graphs=512, seed=SEED_BASE + 4):
    """Per-graph recipes of the batched configuration (512 independent graphs)."""
    ss = np.random.SeedSequence(seed)
    r = np.random.default_rng(ss.spawn(1)[0])
    out = []
    for i in range(n_graphs):
        G = int(round(10 ** r.uniform(np.log10(0.2e6), np.log10(20e6))))
        out.append(dict(G=G, cov=float(r.uniform(10, 40)), mean_len=10_000, sd_len=3_000,
                        err=0.0, extra_rate=float(r.uniform(0.005, 0.03)), repeats=None, P=64,
                        name="batch-%d" % i, seed=int(seed * 1000 + i)))
    return out


def batch_graphs(n_graphs=512, seed=SEED_BASE + 4, only=None):
    ps = batch_params(n_graphs, seed)
    idx = range(n_graphs) if only is None else only
    return [simulate(**ps[i]) for i in idx]


def request_params(n_req, seed=SEED_BASE + 5):
    """Recipes of serving requests: genome 1-100 Mbp log-uniform, 15-30x."""
    ss = np.random.SeedSequence(seed)
    r = np.random.default_rng(ss.spawn(1)[0])
    out = []
    for i in range(n_req):
        G = int(round(10 ** r.uniform(6, 8)))
        out.append(dict(G=G, cov=float(r.uniform(15, 30)), mean_len=12_000, sd_len=4_000,
                        err=0.0, extra_rate=float(r.uniform(0.01, 0.02)), repeats=None, P=64,
                        name="req-%d" % i, seed=int(seed * 1000 + i)))
    return out


# ----------------------------------------------------------------------------
# Alignment coordinates per entry (what an aligner reports for each overlap)
# ----------------------------------------------------------------------------

def with_alignment_ends(g: StringGraph, rng=None, max_clip: int = 0) -> StringGraph:
    """A copy of g with explicit per-entry alignment coordinates.

    For entry (u, v) the walk goes along u then v; pre is the stored index of
    the last base of u before the aligned region and post the stored index of
    the first aligned base of v, each counted in the direction the walk takes
    its read (strand bits s, d).  An x-drop alignment may start late: each
    undirected overlap gets clips (x, y) with x + y < ovl, x applied at the
    start of the overlap as walked u -> v and y as walked v -> u (the twin
    entry), so both walks describe the same shortened alignment.  With
    max_clip = 0 the aligned region is the whole overlap."""
    import copy
    rng = rng if rng is not None else np.random.default_rng(0)
    h = copy.copy(g)
    pre = np.zeros(g.m, np.uint32)
    post = np.zeros(g.m, np.uint32)
    src = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.row_ptr))
    clip = {}
    for e in range(g.m):
        u, v = int(src[e]), int(g.col[e])
        key = (min(u, v), max(u, v))
        ov = int(g.ovl[e])
        if key not in clip:
            lim = min(max_clip, (ov - 1) // 2)
            clip[key] = (int(rng.integers(0, lim + 1)), int(rng.integers(0, lim + 1)))
        x = clip[key][0] if u < v else clip[key][1]
        s, d = int(g.strand[e]) & 1, (int(g.strand[e]) >> 1) & 1
        lu, lv = int(g.read_len[u]), int(g.read_len[v])
        # in walking coordinates the overlap starts at lu - ov in u and at 0 in v
        w_pre = lu - ov + x - 1
        w_post = x
        pre[e] = w_pre if s == 0 else lu - 1 - w_pre
        post[e] = w_post if d == 0 else lv - 1 - w_post
    h.pre, h.post = pre, post
    h.meta = dict(g.meta, alignment_clip=max_clip)
    return h


# ----------------------------------------------------------------------------
# Adversarial tiny graphs (cycles, same-end joins, singletons, many bins)
# ----------------------------------------------------------------------------

def adversarial(rng, n_max=12, len_lo=1, len_hi=40):
    """Tiny random valid graph with arbitrary structure and random bits.

    Unlike the genome simulator this draws topology directly, so cycles,
    same-end joins, branch vertices, isolated reads, 2-read chains, reads of
    length 1 and overlaps of length len-1 all occur."""
    n = int(rng.integers(1, n_max + 1))
    lens = rng.integers(len_lo, len_hi + 1, size=n)
    reads = [rng.integers(0, 4, size=int(L), dtype=np.uint8) for L in lens]
    edges = []
    seen = set()
    mode = rng.integers(0, 3)
    if mode == 0:                      # random sparse graph
        k = int(rng.integers(0, 2 * n + 1))
        for _ in range(k):
            x, y = (int(t) for t in rng.integers(0, n, size=2))
            if x != y and (min(x, y), max(x, y)) not in seen:
                seen.add((min(x, y), max(x, y)))
                edges.append((x, y))
    else:                              # disjoint chains and cycles, plus a few extras
        perm = rng.permutation(n).tolist()
        i = 0
        while i < n:
            q = int(rng.integers(1, n - i + 1))
            grp = perm[i: i + q]
            for a_, b_ in zip(grp[:-1], grp[1:]):
                seen.add((min(a_, b_), max(a_, b_)))
                edges.append((a_, b_))
            if q >= 3 and rng.random() < 0.5:
                seen.add((min(grp[0], grp[-1]), max(grp[0], grp[-1])))
                edges.append((grp[-1], grp[0]))
            i += q
        if mode == 2:
            for _ in range(int(rng.integers(0, 3))):
                x, y = (int(t) for t in rng.integers(0, n, size=2))
                if x != y and (min(x, y), max(x, y)) not in seen:
                    seen.add((min(x, y), max(x, y)))
                    edges.append((x, y))
    out = []
    for x, y in edges:
        hi = int(min(lens[x], lens[y])) - 1
        if hi < 1:
            continue
        out.append((x, y, int(rng.integers(1, hi + 1)), int(rng.integers(0, 2)),
                    int(rng.integers(0, 2))))
    return graph_from_edges(reads, out, meta={"name": "adversarial"})

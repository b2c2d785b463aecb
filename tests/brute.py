"""Brute-force and string-level checks used to pin the oracle.

These are written independently of the oracle's C code and use different
methods: degree by column counts, components by breadth-first search, chain
layouts by exhaustive simple-path enumeration, contigs by Python string
operations on decoded reads, and LPT optimality by exhaustive search.
"""
from __future__ import annotations

import itertools
from collections import deque

import numpy as np

COMP = {"A": "T", "C": "G", "G": "C", "T": "A"}


def revcomp(s: str) -> str:
    return "".join(COMP[c] for c in reversed(s))


def read_str(g, v) -> str:
    L = int(g.read_len[v])
    o = int(g.read_off[v])
    out = []
    for i in range(o, o + L):
        out.append("ACGT"[(int(g.seq[i // 16]) >> (2 * (i % 16))) & 3])
    return "".join(out)


def entries(g):
    """Directed entries as a dict (u, v) -> (ovl, s, d, entry index)."""
    out = {}
    for u in range(g.n):
        for j in range(int(g.row_ptr[u]), int(g.row_ptr[u + 1])):
            b = int(g.strand[j])
            out[(u, int(g.col[j]))] = (int(g.ovl[j]), b & 1, (b >> 1) & 1, j)
    return out


def bf_mask(g):
    deg = np.bincount(np.asarray(g.col, dtype=np.int64), minlength=g.n)   # column counts
    branch = set(int(v) for v in np.nonzero(deg >= 3)[0])
    kept = set()
    for (u, v) in entries(g):
        if u not in branch and v not in branch:
            kept.add((u, v))
    return deg, branch, kept


def bf_components(n, kept):
    adj = [[] for _ in range(n)]
    for (u, v) in kept:
        adj[u].append(v)
    label = [-1] * n
    for s in range(n):
        if label[s] >= 0:
            continue
        seen = [s]
        label[s] = s
        dq = deque([s])
        while dq:
            x = dq.popleft()
            for y in adj[x]:
                if label[y] < 0:
                    label[y] = s
                    seen.append(y)
                    dq.append(y)
        m = min(seen)
        for x in seen:
            label[x] = m
    return np.array(label, dtype=np.int64), adj


def hamiltonian_paths(verts, adj):
    """All simple paths visiting every vertex of the component (tiny only)."""
    vs = set(verts)
    q = len(verts)
    out = []

    def rec(path, seen):
        if len(path) == q:
            out.append(list(path))
            return
        for y in adj[path[-1]]:
            if y in vs and y not in seen:
                seen.add(y)
                path.append(y)
                rec(path, seen)
                path.pop()
                seen.discard(y)

    for s in verts:
        rec([s], {s})
    return out


def contig_from_walk(g, walk, ent):
    """Contig of a walk by string operations: orient each read, keep the part
    of each read that precedes its overlap with the next read, keep the last
    read whole.  Returns (contig, orientations, same_end_join)."""
    if len(walk) == 1:
        return read_str(g, walk[0]), [0], False
    orient = []
    pieces = []
    sej = False
    for k, v in enumerate(walk):
        if k == 0:
            o = ent[(walk[0], walk[1])][1]
        else:
            o = ent[(walk[k - 1], v)][2]
        orient.append(o)
        s = read_str(g, v)
        s = revcomp(s) if o else s
        if k + 1 < len(walk):
            ov, sbit, _, _ = ent[(v, walk[k + 1])]
            if sbit != o:
                sej = True
            pieces.append(s[: len(s) - ov])
        else:
            pieces.append(s)
    return "".join(pieces), orient, sej


def lpt_opt(sizes, P):
    """Optimal makespan by exhaustive assignment (tiny instances)."""
    best = None
    for assign in itertools.product(range(P), repeat=len(sizes)):
        loads = [0] * P
        for s, b in zip(sizes, assign):
            loads[b] += s
        mk = max(loads)
        if best is None or mk < best:
            best = mk
    return best if best is not None else 0


def graham_family(P):
    """Graham's tight instance for LPT: 2P-1, 2P-1, 2P-2, 2P-2, ..., P+1, P+1, P, P, P."""
    out = []
    for x in range(2 * P - 1, P, -1):
        out += [x, x]
    out += [P, P, P]
    return out

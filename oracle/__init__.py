"""CPU oracle for the contig-generation path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  It loads ``liboracle.so`` (plain C, built from ``cgoracle.c`` by
gcc) and runs the paper's Algorithm 2 step by step on host numpy arrays.  It
shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_LIB = None

SINGLE, PATH, CYCLE = 0, 1, 2
CIRCULAR, SAME_END_JOIN, SINGLE_READ = 1, 2, 4


def build(force: bool = False) -> str:
    src = os.path.join(_HERE, "cgoracle.c")
    hdr = os.path.join(_HERE, "cgoracle.h")
    newest = max(os.path.getmtime(src), os.path.getmtime(hdr))
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < newest:
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               src, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    if _LIB is None:
        _LIB = ctypes.CDLL(build())
        for name in ("cgo_validate", "cgo_mask", "cgo_components", "cgo_table", "cgo_lpt",
                     "cgo_order", "cgo_induce", "cgo_assemble", "cgo_reduce"):
            getattr(_LIB, name).argtypes = None
        _LIB.cgo_validate.restype = ctypes.c_int64
        _LIB.cgo_table.restype = ctypes.c_int32
        _LIB.cgo_assemble.restype = ctypes.c_int32
        _LIB.cgo_mask.restype = None
        _LIB.cgo_components.restype = None
        _LIB.cgo_lpt.restype = None
        _LIB.cgo_order.restype = None
        _LIB.cgo_induce.restype = None
        _LIB.cgo_reduce.restype = ctypes.c_int64
    return _LIB


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def _i32(x):
    return ctypes.c_int32(int(x))


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _pre_post(g):
    """The graph's explicit pre/post arrays (Section 4.4) as uint32 arrays, or
    None; the caller keeps them referenced while C reads them."""
    pre, post = getattr(g, "pre", None), getattr(g, "post", None)
    if pre is None:
        return None
    return _c(pre, np.uint32), _c(post, np.uint32)


def _pp_args(pp):
    return (ctypes.c_void_p(0), ctypes.c_void_p(0)) if pp is None else (_p(pp[0]), _p(pp[1]))


def validate(g):
    why = np.zeros(1, np.int32)
    pp = _pre_post(g)
    bad = _lib().cgo_validate(_i32(g.n), _i32(g.m), _p(_c(g.row_ptr, np.int32)),
                              _p(_c(g.col, np.int32)), _p(_c(g.ovl, np.uint32)),
                              _p(_c(g.strand, np.uint8)), _p(_c(g.read_len, np.uint32)),
                              _p(_c(g.read_off, np.uint64)), ctypes.c_uint64(g.seq.shape[0]),
                              *_pp_args(pp), _p(why))
    return int(bad), int(why[0])


def mask(n, row_ptr, col):
    flags = np.zeros(max(n, 1), np.uint8)
    counts = np.zeros(2, np.int32)
    _lib().cgo_mask(_i32(n), _p(_c(row_ptr, np.int32)), _p(_c(col, np.int32)), _p(flags),
                    _p(counts))
    return flags[:n], counts


def components(n, row_ptr, col, flags):
    label = np.zeros(max(n, 1), np.int32)
    _lib().cgo_components(_i32(n), _p(_c(row_ptr, np.int32)), _p(_c(col, np.int32)),
                          _p(_c(flags, np.uint8)), _p(label))
    return label[:n]


def table(n, row_ptr, flags, label, min_reads=2):
    k = max(n, 1)
    comp_label = np.zeros(k, np.int32)
    comp_size = np.zeros(k, np.int32)
    comp_kind = np.zeros(k, np.uint8)
    label_comp = np.zeros(k, np.int32)
    n_comp = _lib().cgo_table(_i32(n), _p(_c(row_ptr, np.int32)), _p(_c(flags, np.uint8)),
                              _p(_c(label, np.int32)), _i32(min_reads), _p(comp_label),
                              _p(comp_size), _p(comp_kind), _p(label_comp))
    if n_comp < 0:
        raise RuntimeError("component is neither a path nor a cycle")
    return (comp_label[:n_comp], comp_size[:n_comp], comp_kind[:n_comp], label_comp[:n])


def lpt(weights, comp_label, P):
    nc = len(weights)
    w = np.ascontiguousarray(weights, dtype=np.uint64)
    comp_bin = np.zeros(max(nc, 1), np.int32)
    bin_load = np.zeros(max(P, 1), np.uint64)
    _lib().cgo_lpt(_i32(nc), _p(w), _p(_c(comp_label, np.int32)), _i32(P), _p(comp_bin),
                   _p(bin_load))
    return comp_bin[:nc], bin_load[:P]


def component_weights(g, label, label_comp, comp_size, weight="reads"):
    """LPT weight of each eligible component: its read count (Section 4.3),
    or with weight="bases" the total length of its reads.  Bases weights of
    2^32 or more are outside the library's range and raise ValueError."""
    if weight == "reads":
        return np.asarray(comp_size, np.uint64)
    if weight != "bases":
        raise ValueError("weight must be 'reads' or 'bases'")
    owner = np.asarray(label_comp)[np.asarray(label)] if g.n else np.zeros(0, np.int64)
    keep = owner >= 0
    w = np.zeros(len(comp_size), np.uint64)
    np.add.at(w, owner[keep], g.read_len[keep].astype(np.uint64))
    if len(w) and int(w.max()) >= 1 << 32:
        raise ValueError("a component's bases weight reaches 2^32")
    return w


def order(comp_label, comp_bin, comp_size):
    nc = len(comp_label)
    rank = np.zeros(max(nc, 1), np.int32)
    start = np.zeros(max(nc, 1), np.int32)
    _lib().cgo_order(_i32(nc), _p(_c(comp_label, np.int32)), _p(_c(comp_bin, np.int32)),
                     _p(_c(comp_size, np.int32)), _p(rank), _p(start))
    return rank[:nc], start[:nc]


def induce(g, flags, label, parts, P):
    n = g.n
    k = max(n, 1)
    perm = np.zeros(k, np.int32)
    bin_vptr = np.zeros(P + 1, np.int32)
    loc_row_ptr = np.zeros(n + 1, np.int32)
    loc_col = np.zeros(2 * k, np.int32)
    loc_eid = np.zeros(2 * k, np.int32)
    sizes = np.zeros(2, np.int32)
    _lib().cgo_induce(_i32(n), _p(_c(g.row_ptr, np.int32)), _p(_c(g.col, np.int32)),
                      _p(_c(flags, np.uint8)), _p(_c(label, np.int32)),
                      _i32(len(parts["comp_label"])), _p(_c(parts["label_comp"], np.int32)),
                      _p(_c(parts["comp_bin"], np.int32)), _p(_c(parts["comp_start"], np.int32)),
                      _i32(P), _p(_c(parts["comp_size"], np.int32)), _p(perm), _p(bin_vptr),
                      _p(loc_row_ptr), _p(loc_col), _p(loc_eid), _p(sizes))
    n_e, m_e = int(sizes[0]), int(sizes[1])
    return dict(perm=perm[:n_e], bin_vptr=bin_vptr, loc_row_ptr=loc_row_ptr[:n_e + 1],
                loc_col=loc_col[:m_e], loc_eid=loc_eid[:m_e], n_e=n_e, m_e=m_e)


def assemble(g, parts, local, cap_words=None):
    nc = len(parts["comp_label"])
    k = max(nc, 1)
    n_e = local["n_e"]
    if cap_words is None:
        cap_words = int(g.seq.shape[0]) + nc
    recs = dict(label=np.zeros(k, np.int32), bin=np.zeros(k, np.int32),
                start=np.zeros(k, np.int32), n_reads=np.zeros(k, np.int32),
                len=np.zeros(k, np.uint64), base_off=np.zeros(k, np.uint64),
                cflags=np.zeros(k, np.uint32), layout_off=np.zeros(k, np.int32))
    layout_vid = np.zeros(max(n_e, 1), np.int32)
    layout_rev = np.zeros(max(n_e, 1), np.uint8)
    bases = np.zeros(max(cap_words, 1), np.uint32)
    total = np.zeros(1, np.uint64)
    pp = _pre_post(g)
    rc = _lib().cgo_assemble(
        _i32(g.n), _p(_c(g.row_ptr, np.int32)), _p(_c(g.col, np.int32)), _p(_c(g.ovl, np.uint32)),
        _p(_c(g.strand, np.uint8)), _p(_c(g.read_len, np.uint32)), _p(_c(g.read_off, np.uint64)),
        _p(_c(g.seq, np.uint32)), *_pp_args(pp), _i32(nc), _p(_c(parts["comp_label"], np.int32)),
        _p(_c(parts["comp_size"], np.int32)), _p(_c(parts["comp_kind"], np.uint8)),
        _p(_c(parts["comp_bin"], np.int32)), _p(_c(parts["comp_rank"], np.int32)),
        _p(_c(parts["comp_start"], np.int32)), _p(_c(local["perm"], np.int32)),
        _p(_c(local["loc_row_ptr"], np.int32)), _p(_c(local["loc_col"], np.int32)),
        _p(_c(local["loc_eid"], np.int32)), _p(recs["label"]), _p(recs["bin"]),
        _p(recs["start"]), _p(recs["n_reads"]), _p(recs["len"]), _p(recs["base_off"]),
        _p(recs["cflags"]), _p(recs["layout_off"]), _p(layout_vid), _p(layout_rev), _p(bases),
        ctypes.c_uint64(cap_words), _p(total))
    if rc == -1:
        raise RuntimeError("walk did not visit a whole component")
    out = {key: v[:nc] for key, v in recs.items()}
    out.update(layout_vid=layout_vid[:n_e], layout_rev=layout_rev[:n_e],
               total_words=int(total[0]), status=int(rc))
    out["bases"] = bases[: int(total[0])] if rc == 0 else bases[:0]
    return out


def run(g, P, min_reads=2, timings=None, weight="reads"):
    """All five steps of Algorithm 2 on one graph; returns a dict of outputs.

    weight: "reads" (the paper's component size) or "bases" (total read
    length) for GreedyPartitioning.  If ``timings`` is a dict, per-step wall
    times (seconds) are stored in it."""
    t = time.perf_counter
    t0 = t()
    flags, counts = mask(g.n, g.row_ptr, g.col)
    t1 = t()
    label = components(g.n, g.row_ptr, g.col, flags)
    t2 = t()
    comp_label, comp_size, comp_kind, label_comp = table(g.n, g.row_ptr, flags, label, min_reads)
    weights = component_weights(g, label, label_comp, comp_size, weight)
    comp_bin, bin_load = lpt(weights, comp_label, P)
    comp_rank, comp_start = order(comp_label, comp_bin, comp_size)
    t3 = t()
    parts = dict(comp_label=comp_label, comp_size=comp_size, comp_kind=comp_kind,
                 comp_bin=comp_bin, comp_rank=comp_rank, comp_start=comp_start,
                 bin_load=bin_load, label_comp=label_comp, n_comp=len(comp_label))
    local = induce(g, flags, label, parts, P)
    t4 = t()
    contigs = assemble(g, parts, local)
    t5 = t()
    if timings is not None:
        timings.update(mask=t1 - t0, components=t2 - t1, partition=t3 - t2, induce=t4 - t3,
                       assemble=t5 - t4, total=t5 - t0)
    return dict(flags=flags, counts=counts, label=label, parts=parts, local=local,
                contigs=contigs)


def contig_codes(contigs, k):
    """Base codes (uint8) of contig k from the packed output (test helper)."""
    L = int(contigs["len"][k])
    off = int(contigs["base_off"][k])
    idx = off + np.arange(L, dtype=np.int64)
    return ((contigs["bases"][idx >> 4] >> (2 * (idx & 15)).astype(np.uint32)) & 3).astype(np.uint8)


def reduce(r, fuzz=0):
    """Prune(IsContainedRead) and TransitiveReduction (Algorithm 1; Section 2)
    of an overlap graph r (fields as a string graph's).  Returns (contained
    u8[n], kept u8[m], the reduced graph as a copy of r with its CSR arrays
    replaced)."""
    import dataclasses
    n = r.n
    m = int(r.row_ptr[n]) if n else 0
    row_ptr, col = _c(r.row_ptr, np.int32), _c(r.col, np.int32)
    ovl, strand = _c(r.ovl, np.uint32), _c(r.strand, np.uint8)
    read_len = _c(r.read_len, np.uint32)
    contained = np.zeros(max(n, 1), np.uint8)
    kept = np.zeros(max(m, 1), np.uint8)
    s_row_ptr = np.zeros(n + 1, np.int32)
    s_col = np.zeros(max(m, 1), np.int32)
    s_ovl = np.zeros(max(m, 1), np.uint32)
    s_strand = np.zeros(max(m, 1), np.uint8)
    ms = _lib().cgo_reduce(_i32(n), _p(row_ptr), _p(col), _p(ovl), _p(strand), _p(read_len),
                           ctypes.c_uint32(int(fuzz)), _p(contained), _p(kept), _p(s_row_ptr),
                           _p(s_col), _p(s_ovl), _p(s_strand))
    s = dataclasses.replace(r, m=int(ms), row_ptr=s_row_ptr, col=s_col[:ms].copy(),
                            ovl=s_ovl[:ms].copy(), strand=s_strand[:ms].copy(), pre=None,
                            post=None)
    return contained[:n], kept[:m], s

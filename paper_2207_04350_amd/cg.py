"""ctypes binding of libcg (include/cg.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch provides device memory and streams.  Importing this module does not
require a GPU; calling into the library does, and a missing libcg.so raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcg.so")
_LIB = None

CG_OK, CG_EINVAL, CG_ENOMEM, CG_EHIP, CG_ECAPACITY, CG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
KIND_SINGLE, KIND_PATH, KIND_CYCLE = 0, 1, 2
CONTIG_CIRCULAR, CONTIG_SAME_END_JOIN, CONTIG_SINGLE = 1, 2, 4
STATUS_BASES_OVERFLOW = 1
STATUS_SCAN_STALLED = 2

_vp = ctypes.c_void_p


class CgGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("m", ctypes.c_int32), ("row_ptr", _vp), ("col", _vp),
                ("ovl", _vp), ("strand", _vp), ("read_len", _vp), ("read_off", _vp),
                ("seq", _vp), ("seq_words", ctypes.c_uint64), ("pre", _vp), ("post", _vp)]


class CgParts(ctypes.Structure):
    _fields_ = [("comp_label", _vp), ("comp_size", _vp), ("comp_kind", _vp), ("comp_bin", _vp),
                ("comp_rank", _vp), ("comp_start", _vp), ("bin_load", _vp),
                ("label_comp", _vp), ("d_n_comp", _vp)]


class CgLocal(ctypes.Structure):
    _fields_ = [("perm", _vp), ("bin_vptr", _vp), ("loc_row_ptr", _vp), ("loc_col", _vp),
                ("loc_eid", _vp), ("d_sizes", _vp)]


class CgContigs(ctypes.Structure):
    _fields_ = [("label", _vp), ("bin", _vp), ("start", _vp), ("n_reads", _vp), ("len", _vp),
                ("base_off", _vp), ("cflags", _vp), ("layout_off", _vp), ("layout_vid", _vp),
                ("layout_rev", _vp), ("bases", _vp), ("cap_words", ctypes.c_uint64),
                ("d_total_words", _vp)]


class CgSizes(ctypes.Structure):
    _fields_ = [("scratch", ctypes.c_uint64), ("graph", ctypes.c_uint64),
                ("outputs", ctypes.c_uint64)]


class CgJob(ctypes.Structure):
    _fields_ = [("g", CgGraph), ("P", ctypes.c_int32), ("min_reads", ctypes.c_int32),
                ("weight", ctypes.c_int32), ("flags", _vp), ("d_counts", _vp), ("label", _vp), ("parts", CgParts),
                ("local", CgLocal), ("contigs", CgContigs)]


class CgBatchParams(ctypes.Structure):
    _fields_ = [("vertex_tile", ctypes.c_int32), ("copy_block", ctypes.c_int32),
                ("persist_blocks", ctypes.c_int32)]


class CgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libcg error %d: %s" % (code, msg))
        self.code = code


def lib():
    """The loaded libcg.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcg.so is not built (run __graft_entry__.build() or "
                               "python -m paper_2207_04350_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        L.cg_last_error.restype = ctypes.c_char_p
        L.cg_ctx_create.argtypes = [ctypes.c_int, ctypes.c_size_t, P(_vp)]
        L.cg_ctx_destroy.argtypes = [_vp]
        L.cg_footprint.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                   ctypes.c_int32, ctypes.c_int32, P(CgSizes)]
        L.cg_ctx_status.argtypes = [_vp, _vp, P(ctypes.c_uint32), ctypes.c_int]
        L.cg_validate.argtypes = [_vp, P(CgGraph), _vp, _vp]
        L.cg_mask_branches.argtypes = [_vp, P(CgGraph), _vp, _vp, _vp]
        L.cg_components.argtypes = [_vp, P(CgGraph), _vp, _vp, _vp]
        L.cg_partition.argtypes = [_vp, P(CgGraph), _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, P(CgParts), _vp]
        L.cg_induce.argtypes = [_vp, P(CgGraph), _vp, _vp, P(CgParts), ctypes.c_int32,
                                P(CgLocal), _vp]
        L.cg_assemble.argtypes = [_vp, P(CgGraph), P(CgParts), P(CgLocal), ctypes.c_int32,
                                  P(CgContigs), _vp]
        L.cg_ctx_profile.argtypes = [_vp, ctypes.c_int32]
        L.cg_ctx_profile_read.argtypes = [_vp, ctypes.c_int32, P(ctypes.c_char_p),
                                          P(ctypes.c_int64), P(ctypes.c_double),
                                          P(ctypes.c_int32), P(ctypes.c_int64)]
        L.cg_reduce.argtypes = [_vp, P(CgGraph), ctypes.c_uint32, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp]
        L.cg_contig_generation_noalloc.argtypes = [P(CgGraph), ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.c_int32, _vp, _vp, _vp, P(CgParts),
                                                   P(CgLocal), P(CgContigs), _vp, _vp]
        L.cg_batch_create.argtypes = [_vp, ctypes.c_int32, P(CgJob), P(CgBatchParams), P(_vp)]
        L.cg_batch_run.argtypes = [_vp, _vp]
        L.cg_batch_bytes.argtypes = [ctypes.c_int32, P(CgJob), P(CgBatchParams),
                                     P(ctypes.c_uint64)]
        L.cg_batch_create_empty.argtypes = [_vp, ctypes.c_uint64, P(CgBatchParams), P(_vp)]
        L.cg_batch_plan.argtypes = [_vp, ctypes.c_int32, P(CgJob), _vp]
        L.cg_job_outputs.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, _vp,
                                     P(ctypes.c_uint64), P(CgJob)]
        L.cg_batch_counts.argtypes = [_vp, _vp, _vp]
        L.cg_batch_pack.argtypes = [_vp, _vp, _vp, ctypes.c_uint64, _vp]
        L.cg_batch_capture.argtypes = [_vp, _vp]
        L.cg_batch_launch.argtypes = [_vp, _vp]
        L.cg_batch_destroy.argtypes = [_vp]
        for name in ("cg_batch_create", "cg_batch_run", "cg_batch_bytes", "cg_batch_create_empty",
                     "cg_batch_plan", "cg_batch_capture", "cg_batch_launch", "cg_job_outputs",
                     "cg_batch_counts", "cg_batch_pack",
                     "cg_batch_destroy", "cg_ctx_profile", "cg_ctx_profile_read",
                     "cg_ctx_create", "cg_ctx_destroy", "cg_footprint", "cg_ctx_status",
                     "cg_validate", "cg_mask_branches", "cg_components", "cg_partition",
                     "cg_induce", "cg_assemble", "cg_reduce", "cg_contig_generation_noalloc"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB


def _check(rc):
    if rc != CG_OK:
        raise CgError(rc, lib().cg_last_error().decode(errors="replace"))


def _ptr(t):
    return _vp(t.data_ptr()) if t is not None else _vp(0)


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return _vp(s.cuda_stream)


def sizes(n, m, seq_words, P, coords=False):
    """cg_footprint: device bytes of a graph of n reads, m entries and
    seq_words packed words at P bins, as {"scratch", "graph", "outputs"}."""
    out = CgSizes()
    _check(lib().cg_footprint(int(n), int(m), int(seq_words), int(P), int(bool(coords)),
                              ctypes.byref(out)))
    return {"scratch": int(out.scratch), "graph": int(out.graph), "outputs": int(out.outputs)}


def footprint(n, m, P):
    """Context scratch bytes for graphs of up to n reads, m entries, P bins."""
    return sizes(n, m, 0, P)["scratch"]


class Context:
    """A cg_ctx: device scratch sized by footprint(n, m, P)."""

    def __init__(self, device=0, scratch_bytes=0):
        self.handle = _vp(0)
        self.device = device
        self.scratch_bytes = int(scratch_bytes)
        _check(lib().cg_ctx_create(int(device), self.scratch_bytes, ctypes.byref(self.handle)))

    @classmethod
    def for_graph(cls, n, m, P, device=0, slack=1.0):
        return cls(device, int(footprint(n, m, P) * slack))

    def status(self, stream=None, clear=True):
        s = ctypes.c_uint32(0)
        _check(lib().cg_ctx_status(self.handle, _stream(stream), ctypes.byref(s), int(clear)))
        return int(s.value)

    def profile(self, max_launches):
        """Bracket each kernel launch with HIP events (0 switches it off)."""
        _check(lib().cg_ctx_profile(self.handle, int(max_launches)))

    def profile_read(self):
        """{kernel name: (launches, total ms)} since the last read."""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        launches = (ctypes.c_int64 * cap)()
        ms = (ctypes.c_double * cap)()
        nk = ctypes.c_int32(0)
        dropped = ctypes.c_int64(0)
        _check(lib().cg_ctx_profile_read(self.handle, cap, names, launches, ms,
                                         ctypes.byref(nk), ctypes.byref(dropped)))
        out = {names[i].decode(): (int(launches[i]), float(ms[i])) for i in range(nk.value)}
        if dropped.value:
            out["_dropped"] = (int(dropped.value), 0.0)
        return out

    def close(self):
        if self.handle and self.handle.value:
            _check(lib().cg_ctx_destroy(self.handle))
            self.handle = _vp(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Device-resident inputs and outputs (torch tensors + the C structs)
# ---------------------------------------------------------------------------

def _dev(a, dtype, device):
    """numpy array -> device tensor; unsigned types travel as same-width signed."""
    import torch
    a = np.ascontiguousarray(a)
    view = {np.dtype(np.uint32): np.int32, np.dtype(np.uint64): np.int64}.get(a.dtype)
    if view is not None:
        a = a.view(view)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device)


class DeviceGraph:
    """A string graph resident in device memory."""

    def __init__(self, g, device="cuda"):
        import torch
        self.n, self.m = int(g.n), int(g.m)
        self.row_ptr = _dev(g.row_ptr.astype(np.int32), None, device)
        self.col = _dev(g.col.astype(np.int32) if g.m else np.zeros(1, np.int32), None, device)
        self.ovl = _dev(g.ovl.astype(np.uint32) if g.m else np.zeros(1, np.uint32), None, device)
        self.strand = _dev(g.strand.astype(np.uint8) if g.m else np.zeros(1, np.uint8), None,
                           device)
        self.read_len = _dev(g.read_len.astype(np.uint32) if g.n else np.zeros(1, np.uint32),
                             None, device)
        self.read_off = _dev(g.read_off.astype(np.uint64) if g.n else np.zeros(1, np.uint64),
                             None, device)
        self.seq = _dev(g.seq.astype(np.uint32), None, device)
        self.seq_words = int(g.seq.shape[0])
        # optional per-entry pre/post (Section 4.4), else derived from ovl
        pre, post = getattr(g, "pre", None), getattr(g, "post", None)
        self.pre = self.post = None
        if pre is not None:
            z = lambda a: a.astype(np.uint32) if g.m else np.zeros(1, np.uint32)
            self.pre, self.post = _dev(z(pre), None, device), _dev(z(post), None, device)
        self.struct = CgGraph(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.ovl),
                              _ptr(self.strand), _ptr(self.read_len), _ptr(self.read_off),
                              _ptr(self.seq), self.seq_words, _ptr(self.pre), _ptr(self.post))
        self.device = torch.device(device)


    @classmethod
    def from_tensors(cls, n, m, t, seq_words, device="cuda"):
        """A resident graph from device tensors already in place (keys row_ptr,
        col, ovl, strand, read_len, read_off, seq and optionally pre, post;
        unsigned arrays as same-width signed tensors)."""
        import torch
        self = cls.__new__(cls)
        self.n, self.m = int(n), int(m)
        for k in ("row_ptr", "col", "ovl", "strand", "read_len", "read_off", "seq"):
            setattr(self, k, t[k])
        self.pre, self.post = t.get("pre"), t.get("post")
        self.seq_words = int(seq_words)
        self.struct = CgGraph(self.n, self.m, _ptr(self.row_ptr), _ptr(self.col), _ptr(self.ovl),
                              _ptr(self.strand), _ptr(self.read_len), _ptr(self.read_off),
                              _ptr(self.seq), self.seq_words, _ptr(self.pre), _ptr(self.post))
        self.device = torch.device(device)
        return self


class Outputs:
    """Every output buffer of the five calls for one graph (upper-bound sized)."""

    def __init__(self, n, P, cap_words, device="cuda"):
        import torch
        k = max(int(n), 1)
        i32, i64, u8 = torch.int32, torch.int64, torch.uint8
        e = lambda size, dt: torch.empty(size, dtype=dt, device=device)
        self.n, self.P, self.cap_words = int(n), int(P), int(cap_words)
        self.flags = e(k, u8)
        self.counts = e(2, i32)
        self.label = e(k, i32)
        self.comp_label, self.comp_size, self.comp_kind = e(k, i32), e(k, i32), e(k, u8)
        self.comp_bin, self.comp_rank, self.comp_start = e(k, i32), e(k, i32), e(k, i32)
        self.bin_load = e(P, i64)
        self.label_comp = e(k, i32)
        self.n_comp = e(1, i32)
        self.perm, self.bin_vptr = e(k, i32), e(P + 1, i32)
        self.loc_row_ptr, self.loc_col, self.loc_eid = e(k + 1, i32), e(2 * k, i32), e(2 * k, i32)
        self.sizes = e(2, i32)
        self.c_label, self.c_bin, self.c_start, self.c_nreads = (e(k, i32), e(k, i32), e(k, i32),
                                                                 e(k, i32))
        self.c_len, self.c_base_off = e(k, i64), e(k, i64)
        self.c_flags, self.c_layout_off = e(k, i32), e(k, i32)
        self.layout_vid, self.layout_rev = e(k, i32), e(k, u8)
        self.bases = e(max(int(cap_words), 1), i32)
        self.total_words = e(1, i64)
        self.parts = CgParts(_ptr(self.comp_label), _ptr(self.comp_size), _ptr(self.comp_kind),
                             _ptr(self.comp_bin), _ptr(self.comp_rank), _ptr(self.comp_start),
                             _ptr(self.bin_load), _ptr(self.label_comp), _ptr(self.n_comp))
        self.local = CgLocal(_ptr(self.perm), _ptr(self.bin_vptr), _ptr(self.loc_row_ptr),
                             _ptr(self.loc_col), _ptr(self.loc_eid), _ptr(self.sizes))
        self.contigs = CgContigs(_ptr(self.c_label), _ptr(self.c_bin), _ptr(self.c_start),
                                 _ptr(self.c_nreads), _ptr(self.c_len), _ptr(self.c_base_off),
                                 _ptr(self.c_flags), _ptr(self.c_layout_off),
                                 _ptr(self.layout_vid), _ptr(self.layout_rev), _ptr(self.bases),
                                 int(cap_words), _ptr(self.total_words))


# ---------------------------------------------------------------------------
# The calls (same names as the C ABI)
# ---------------------------------------------------------------------------

def validate(ctx, dg, d_bad, stream=None):
    _check(lib().cg_validate(ctx.handle, ctypes.byref(dg.struct), _ptr(d_bad), _stream(stream)))


def mask_branches(ctx, dg, flags, d_counts, stream=None):
    _check(lib().cg_mask_branches(ctx.handle, ctypes.byref(dg.struct), _ptr(flags),
                                  _ptr(d_counts), _stream(stream)))


def components(ctx, dg, flags, label, stream=None):
    _check(lib().cg_components(ctx.handle, ctypes.byref(dg.struct), _ptr(flags), _ptr(label),
                               _stream(stream)))


class Reduced:
    """Outputs of cg_reduce for an overlap graph of n reads and m entries."""

    def __init__(self, n, m, device="cuda"):
        import torch
        e = lambda size, dt: torch.empty(max(int(size), 1), dtype=dt, device=device)
        self.n, self.m_cap = int(n), int(m)
        self.contained = e(n, torch.uint8)
        self.kept = e(m, torch.uint8)
        self.row_ptr = torch.empty(int(n) + 1, dtype=torch.int32, device=device)
        self.col, self.ovl, self.strand = e(m, torch.int32), e(m, torch.int32), e(m, torch.uint8)
        self.d_m = e(1, torch.int32)

    def graph(self, r_dg):
        """The string graph as a resident graph (reads of r_dg); reads the
        device entry count."""
        m = int(self.d_m.item())
        t = dict(row_ptr=self.row_ptr, col=self.col, ovl=self.ovl, strand=self.strand,
                 read_len=r_dg.read_len, read_off=r_dg.read_off, seq=r_dg.seq)
        return DeviceGraph.from_tensors(self.n, m, t, r_dg.seq_words, r_dg.device)


def reduce(ctx, r_dg, out, fuzz=0, stream=None):
    """cg_reduce: contained-read pruning and transitive reduction of the
    overlap graph r_dg into `out` (a Reduced)."""
    _check(lib().cg_reduce(ctx.handle, ctypes.byref(r_dg.struct), ctypes.c_uint32(int(fuzz)),
                           _ptr(out.contained), _ptr(out.kept), _ptr(out.row_ptr), _ptr(out.col),
                           _ptr(out.ovl), _ptr(out.strand), _ptr(out.d_m), _stream(stream)))


WEIGHT_READS, WEIGHT_BASES = 0, 1


def _weight(w):
    return {"reads": WEIGHT_READS, "bases": WEIGHT_BASES}.get(w, w)


def partition(ctx, dg, flags, label, P, min_reads, parts, stream=None, weight="reads"):
    """GreedyPartitioning; weight "reads" (Section 4.3) or "bases"."""
    _check(lib().cg_partition(ctx.handle, ctypes.byref(dg.struct), _ptr(flags), _ptr(label),
                              int(P), int(min_reads), int(_weight(weight)), ctypes.byref(parts),
                              _stream(stream)))


def induce(ctx, dg, flags, label, parts, P, local, stream=None):
    _check(lib().cg_induce(ctx.handle, ctypes.byref(dg.struct), _ptr(flags), _ptr(label),
                           ctypes.byref(parts), int(P), ctypes.byref(local), _stream(stream)))


def assemble(ctx, dg, parts, local, P, contigs, stream=None):
    _check(lib().cg_assemble(ctx.handle, ctypes.byref(dg.struct), ctypes.byref(parts),
                             ctypes.byref(local), int(P), ctypes.byref(contigs),
                             _stream(stream)))


def run_path(ctx, dg, out, P, min_reads=2, stream=None, weight="reads"):
    """Enqueue all five steps of Algorithm 2 for one resident graph."""
    mask_branches(ctx, dg, out.flags, out.counts, stream)
    components(ctx, dg, out.flags, out.label, stream)
    partition(ctx, dg, out.flags, out.label, P, min_reads, out.parts, stream, weight)
    induce(ctx, dg, out.flags, out.label, out.parts, P, out.local, stream)
    assemble(ctx, dg, out.parts, out.local, P, out.contigs, stream)


NOALLOC_SCRATCH_BYTES = 64 << 20


def contig_generation_noalloc(dg, out, P, min_reads=2, stream=None, weight="reads",
                              d_status=None):
    """cg_contig_generation_noalloc: the five steps without a context and
    without allocating (scratch in the library's static device array)."""
    _check(lib().cg_contig_generation_noalloc(
        ctypes.byref(dg.struct), int(P), int(min_reads), int(_weight(weight)), _ptr(out.flags),
        _ptr(out.counts), _ptr(out.label), ctypes.byref(out.parts), ctypes.byref(out.local),
        ctypes.byref(out.contigs), _ptr(d_status), _stream(stream)))


def to_host(out, n):
    """Copy the outputs back, trimmed to their device-side counts, in the same
    dictionary layout the tests use for the oracle."""
    import torch
    torch.cuda.synchronize()
    h = lambda t: t.cpu().numpy()
    nc = int(out.n_comp.item())
    sizes = h(out.sizes)
    n_e, m_e = int(sizes[0]), int(sizes[1])
    tw = int(out.total_words.item())
    parts = dict(comp_label=h(out.comp_label)[:nc], comp_size=h(out.comp_size)[:nc],
                 comp_kind=h(out.comp_kind)[:nc], comp_bin=h(out.comp_bin)[:nc],
                 comp_rank=h(out.comp_rank)[:nc], comp_start=h(out.comp_start)[:nc],
                 bin_load=h(out.bin_load).view(np.uint64), label_comp=h(out.label_comp)[:n],
                 n_comp=nc)
    local = dict(perm=h(out.perm)[:n_e], bin_vptr=h(out.bin_vptr),
                 loc_row_ptr=h(out.loc_row_ptr)[:n_e + 1], loc_col=h(out.loc_col)[:m_e],
                 loc_eid=h(out.loc_eid)[:m_e], n_e=n_e, m_e=m_e)
    contigs = dict(label=h(out.c_label)[:nc], bin=h(out.c_bin)[:nc], start=h(out.c_start)[:nc],
                   n_reads=h(out.c_nreads)[:nc], len=h(out.c_len)[:nc].view(np.uint64),
                   base_off=h(out.c_base_off)[:nc].view(np.uint64),
                   cflags=h(out.c_flags)[:nc].view(np.uint32),
                   layout_off=h(out.c_layout_off)[:nc], layout_vid=h(out.layout_vid)[:n_e],
                   layout_rev=h(out.layout_rev)[:n_e], total_words=tw,
                   bases=(h(out.bases)[:tw].view(np.uint32) if tw <= out.cap_words
                          else np.zeros(0, np.uint32)))
    return dict(flags=h(out.flags)[:n], counts=h(out.counts), label=h(out.label)[:n],
                parts=parts, local=local, contigs=contigs)


def job_outputs_bytes(n, P, cap_words):
    """cg_job_outputs: bytes of one job's outputs carved from one buffer."""
    b = ctypes.c_uint64(0)
    _check(lib().cg_job_outputs(int(n), int(P), int(cap_words), None, ctypes.byref(b), None))
    return int(b.value)


class CarvedOutputs:
    """One job's output buffers inside a larger device buffer (cg_job_outputs):
    only the C pointers, no tensor per buffer."""

    def __init__(self, buf, offset, n, P, cap_words):
        self.buf = buf          # keeps the device buffer alive
        self.n, self.P, self.cap_words = int(n), int(P), int(cap_words)
        self.cjob = CgJob()
        b = ctypes.c_uint64(0)
        _check(lib().cg_job_outputs(self.n, self.P, self.cap_words,
                                    _vp(buf.data_ptr() + int(offset)), ctypes.byref(b),
                                    ctypes.byref(self.cjob)))
        self.nbytes = int(b.value)


# fields of one job's packed results (cg_batch_pack), in order
_PACK_NC = (("len", np.uint64), ("base_off", np.uint64), ("label", np.int32),
            ("bin", np.int32), ("start", np.int32), ("n_reads", np.int32),
            ("cflags", np.uint32), ("layout_off", np.int32))


def unpack_results(packed, row):
    """One job's results from the packed bytes of cg_batch_pack (a uint8
    numpy array) and its row of cg_batch_counts (nc, ne, tw, offset): a dict
    of numpy views."""
    nc, ne, tw, off = (int(x) for x in row)
    out, at = {}, off
    for name, dt in _PACK_NC:
        w = np.dtype(dt).itemsize
        out[name] = packed[at:at + w * nc].view(dt)
        at += w * nc
    out["layout_vid"] = packed[at:at + 4 * ne].view(np.int32)
    at += 4 * ne
    out["bases"] = packed[at:at + 4 * tw].view(np.uint32)
    at += 4 * tw
    out["layout_rev"] = packed[at:at + ne]
    return out


def _job_array(jobs):
    arr = (CgJob * len(jobs))()
    for i, job in enumerate(jobs):
        dg, out, P, mr = job[:4]
        if isinstance(out, CarvedOutputs):
            arr[i] = out.cjob
        arr[i].g = dg.struct
        arr[i].P = int(P)
        arr[i].min_reads = int(mr)
        arr[i].weight = int(_weight(job[4] if len(job) > 4 else "reads"))
        if isinstance(out, CarvedOutputs):
            continue
        arr[i].flags = _ptr(out.flags)
        arr[i].d_counts = _ptr(out.counts)
        arr[i].label = _ptr(out.label)
        arr[i].parts = out.parts
        arr[i].local = out.local
        arr[i].contigs = out.contigs
    return arr


def batch_bytes(jobs, vertex_tile=0):
    """cg_batch_bytes: device bytes a batch of these jobs needs.  A job is a
    (DeviceGraph, Outputs, P, min_reads[, weight]) tuple or, before anything
    is allocated, a (n, m, P[, weight]) tuple of sizes."""
    if jobs and not isinstance(jobs[0][0], DeviceGraph):
        arr = (CgJob * len(jobs))()
        for i, job in enumerate(jobs):
            arr[i].g.n, arr[i].g.m, arr[i].P = int(job[0]), int(job[1]), int(job[2])
            arr[i].weight = int(_weight(job[3] if len(job) > 3 else "reads"))
    else:
        arr = _job_array(jobs)
    out = ctypes.c_uint64(0)
    prm = CgBatchParams(int(vertex_tile), 0, 0)
    _check(lib().cg_batch_bytes(len(jobs), arr, ctypes.byref(prm), ctypes.byref(out)))
    return int(out.value)


class Batch:
    """A cg_batch over resident graphs: `jobs` is a list of (DeviceGraph,
    Outputs, P, min_reads[, weight]).  Keeps the tensors alive while it
    exists.  Batch.empty(ctx, bytes) makes one without jobs, for plan()."""

    def __init__(self, ctx, jobs, vertex_tile=0, copy_block=0, persist_blocks=0):
        self.ctx = ctx
        self._keep = jobs
        prm = CgBatchParams(int(vertex_tile), int(copy_block), int(persist_blocks))
        self.handle = _vp(0)
        if jobs is None:
            return
        _check(lib().cg_batch_create(ctx.handle, len(jobs), _job_array(jobs), ctypes.byref(prm),
                                     ctypes.byref(self.handle)))
        self.params = (vertex_tile, copy_block, persist_blocks)

    @classmethod
    def empty(cls, ctx, nbytes, vertex_tile=0, copy_block=0, persist_blocks=0):
        self = cls(ctx, None)
        prm = CgBatchParams(int(vertex_tile), int(copy_block), int(persist_blocks))
        _check(lib().cg_batch_create_empty(ctx.handle, int(nbytes), ctypes.byref(prm),
                                           ctypes.byref(self.handle)))
        self.params = (vertex_tile, copy_block, persist_blocks)
        self._keep = []
        return self

    def plan(self, jobs, stream=None):
        """cg_batch_plan: replace the jobs (the batch's earlier work must be
        complete)."""
        _check(lib().cg_batch_plan(self.handle, len(jobs), _job_array(jobs), _stream(stream)))
        self._keep = jobs

    def run(self, stream=None):
        _check(lib().cg_batch_run(self.handle, _stream(stream)))

    def counts(self, d_counts, stream=None):
        """cg_batch_counts into d_counts (int64 tensor of 4 n_jobs + 1)."""
        _check(lib().cg_batch_counts(self.handle, _ptr(d_counts), _stream(stream)))

    def pack(self, d_counts, dst, stream=None):
        """cg_batch_pack into dst (a 16-byte aligned device tensor)."""
        _check(lib().cg_batch_pack(self.handle, _ptr(d_counts), _ptr(dst),
                                   dst.numel() * dst.element_size(), _stream(stream)))

    def capture(self, stream):
        _check(lib().cg_batch_capture(self.handle, _stream(stream)))

    def launch(self, stream):
        _check(lib().cg_batch_launch(self.handle, _stream(stream)))

    def close(self):
        if self.handle and self.handle.value:
            _check(lib().cg_batch_destroy(self.handle))
            self.handle = _vp(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

"""Serving form: a continuous-batching loop of contig-generation requests.

Requests (one string graph each) arrive over time.  A request is admitted
when a slot (a cg context with its own stream) is free and its device
footprint fits in the HBM budget next to the requests already on the device;
admitted requests run concurrently on their slots' streams, so a request that
arrives while others are on the GPU starts as soon as a slot and memory free
up.  A request's graph is either uploaded from pinned host memory when the
request is admitted, or already resident: graphs made resident once
(`Server.make_resident`) stay in HBM for the life of the server, charged to
the budget, and requests on them hold only their outputs.  All five steps run
on the device, and the contigs come back to pinned host memory: first the
device-side counts, then exactly the records and bases they name.  Latency is
measured from arrival to the moment the result is in host memory.

The admission core (`Admission`) is plain host logic; `Server` drives it with
real device work.  Every step of the path runs in libcg's kernels.
"""
from __future__ import annotations

import collections
import time

import numpy as np

from . import cg


# ---------------------------------------------------------------------------
# Footprint
# ---------------------------------------------------------------------------

def graph_bytes(n, m, seq_words, pre_post=False):
    """Device bytes of a resident graph (cg_footprint's `graph` figure)."""
    return cg.sizes(n, m, seq_words, 1, pre_post)["graph"]


def output_bytes(n, P, seq_words):
    """Device bytes of one graph's outputs at cap_words = seq_words
    (cg_footprint's `outputs` figure)."""
    return cg.sizes(n, 0, seq_words, P)["outputs"]


def request_footprint(g, P, resident=False):
    """HBM a request holds while it is admitted (its slot's scratch is not
    counted: slots own theirs for the life of the server; nor is a resident
    graph, charged once when it was made resident)."""
    s = cg.sizes(g.n, g.m, g.seq.shape[0], P, getattr(g, "pre", None) is not None)
    return s["outputs"] if resident else s["graph"] + s["outputs"]


# ---------------------------------------------------------------------------
# Admission core (host logic only)
# ---------------------------------------------------------------------------

class Admission:
    """FIFO admission by slots and HBM budget.

    A request is admitted when it is at the head of the queue, a slot is free
    and the footprints of the admitted requests plus its own fit the budget.
    The head is never overtaken, so a large request cannot starve."""

    def __init__(self, slots, budget):
        self.free = list(range(slots))[::-1]
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self.queue = collections.deque()

    def push(self, req_id, footprint):
        if footprint > self.budget:
            raise ValueError("request %r needs %d bytes, above the %d-byte budget"
                             % (req_id, footprint, self.budget))
        self.queue.append((req_id, int(footprint)))

    def admit(self):
        """Admitted (request id, slot) pairs, in arrival order."""
        out = []
        while self.queue and self.free and self.used + self.queue[0][1] <= self.budget:
            rid, fp = self.queue.popleft()
            slot = self.free.pop()
            self.used += fp
            self.peak = max(self.peak, self.used)
            out.append((rid, slot, fp))
        return out

    def release(self, slot, footprint):
        self.used -= footprint
        self.free.append(slot)


# ---------------------------------------------------------------------------
# Requests and the server
# ---------------------------------------------------------------------------

class HostGraph:
    """A string graph in pinned host memory, as requests bring it."""

    def __init__(self, g):
        import torch
        pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        u = lambda a, dt, sdt: a.astype(dt).view(sdt)
        self.graph = g
        self.n, self.m, self.seq_words = g.n, g.m, int(g.seq.shape[0])
        self.t = dict(
            row_ptr=pin(g.row_ptr.astype(np.int32)),
            col=pin(g.col.astype(np.int32) if g.m else np.zeros(1, np.int32)),
            ovl=pin(u(g.ovl, np.uint32, np.int32) if g.m else np.zeros(1, np.int32)),
            strand=pin(g.strand.astype(np.uint8) if g.m else np.zeros(1, np.uint8)),
            read_len=pin(u(g.read_len, np.uint32, np.int32) if g.n else np.zeros(1, np.int32)),
            read_off=pin(u(g.read_off, np.uint64, np.int64) if g.n else np.zeros(1, np.int64)),
            seq=pin(u(g.seq, np.uint32, np.int32)))
        if getattr(g, "pre", None) is not None:
            z = lambda a: u(a, np.uint32, np.int32) if g.m else np.zeros(1, np.int32)
            self.t["pre"], self.t["post"] = pin(z(g.pre)), pin(z(g.post))


class Request:
    """One contig-generation request: a graph in pinned host memory (uploaded
    on admission), or one the server holds resident (`resident=True`), its
    parameters and its arrival time (seconds from the start of the run)."""

    def __init__(self, rid, host, P, min_reads=2, arrival=0.0, resident=False):
        self.rid, self.host, self.P, self.min_reads = rid, host, int(P), int(min_reads)
        self.graph = host.graph
        self.arrival = float(arrival)
        self.resident = bool(resident)
        self.footprint = request_footprint(self.graph, self.P, self.resident)
        self.t_admit = self.t_done = None
        self.result = None


class _Resident:
    """A request's device state while it is admitted."""

    def __init__(self, req, slot, stream, device, dg=None):
        import torch
        self.req, self.slot, self.stream = req, slot, stream
        g = req.graph
        with torch.cuda.stream(stream):
            if dg is None:
                d = {k: v.to(device, non_blocking=True) for k, v in req.host.t.items()}
                dg = cg.DeviceGraph.from_tensors(g.n, g.m, d, int(g.seq.shape[0]), device)
            self.dg = dg
            self.out = cg.Outputs(g.n, req.P, int(g.seq.shape[0]), device)
            self.counts = torch.empty(4, dtype=torch.int64, pin_memory=True)
        self.phase = 0
        self.event = None


class Server:
    """Continuous batching over `slots` concurrent requests within `budget`
    bytes of HBM (default: the device's memory minus `reserve` and the slots'
    scratch).  Slots are sized for graphs of up to max_n reads, max_m entries
    and max_P bins."""

    def __init__(self, max_n, max_m, max_P=64, slots=4, budget=None, reserve=16 << 30,
                 device="cuda", keep_outputs=False):
        import torch
        self.device = torch.device(device)
        self.slots = int(slots)
        self.ctxs = [cg.Context.for_graph(max_n, max_m, max_P, device=self.device.index or 0)
                     for _ in range(self.slots)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.slots)]
        self.max_n, self.max_m, self.max_P = int(max_n), int(max_m), int(max_P)
        if budget is None:
            total = torch.cuda.get_device_properties(self.device).total_memory
            budget = total - reserve - sum(c.scratch_bytes for c in self.ctxs)
        self.budget = int(budget)
        self.keep_outputs = keep_outputs
        self.resident = {}  # id(HostGraph) -> DeviceGraph

    def make_resident(self, host):
        """Upload host (a HostGraph) once; requests with resident=True on it
        then run on this copy.  Its bytes leave the budget for good."""
        import torch
        if id(host) in self.resident:
            return
        g = host.graph
        fp = graph_bytes(g.n, g.m, g.seq.shape[0], getattr(g, "pre", None) is not None)
        if fp > self.budget:
            raise ValueError("graph needs %d bytes, above the %d-byte budget left" % (fp,
                                                                                     self.budget))
        d = {k: v.to(self.device) for k, v in host.t.items()}
        self.resident[id(host)] = cg.DeviceGraph.from_tensors(g.n, g.m, d, int(g.seq.shape[0]),
                                                              self.device)
        torch.cuda.synchronize(self.device)
        self.budget -= fp

    def close(self):
        for c in self.ctxs:
            c.close()
        self.ctxs = []
        self.resident = {}

    # -- per-request device work ------------------------------------------

    def _launch(self, req, slot):
        import torch
        g = req.graph
        if g.n > self.max_n or g.m > self.max_m or req.P > self.max_P:
            raise ValueError("request %r exceeds the slot size" % (req.rid,))
        dg = None
        if req.resident:
            dg = self.resident.get(id(req.host))
            if dg is None:
                raise ValueError("request %r names a graph that is not resident" % (req.rid,))
        r = _Resident(req, slot, self.streams[slot], self.device, dg)
        s = r.stream
        with torch.cuda.stream(s):
            cg.run_path(self.ctxs[slot], r.dg, r.out, req.P, req.min_reads, s)
            o = r.out
            # phase 1: the device-side counts
            cnt = torch.stack([o.n_comp[0].to(torch.int64), o.sizes[0].to(torch.int64),
                               o.total_words[0], o.sizes[1].to(torch.int64)])
            r.counts.copy_(cnt, non_blocking=True)
            r.event = torch.cuda.Event()
            r.event.record(s)
        return r

    def _download(self, r):
        """Phase 2: the records and bases the counts name."""
        import torch
        nc, n_e, tw = (int(x) for x in r.counts[:3].tolist())
        o, s = r.out, r.stream
        pin = lambda t, k: torch.empty(max(k, 1), dtype=t.dtype, pin_memory=True)
        with torch.cuda.stream(s):
            host = {}
            for name, t, k in (("label", o.c_label, nc), ("bin", o.c_bin, nc),
                               ("start", o.c_start, nc), ("n_reads", o.c_nreads, nc),
                               ("len", o.c_len, nc), ("base_off", o.c_base_off, nc),
                               ("cflags", o.c_flags, nc), ("layout_off", o.c_layout_off, nc),
                               ("layout_vid", o.layout_vid, n_e), ("layout_rev", o.layout_rev, n_e),
                               ("bases", o.bases, tw)):
                h = pin(t, k)
                if k:
                    h[:k].copy_(t[:k], non_blocking=True)
                host[name] = (h, k)
            r.host_out = host
            r.event = torch.cuda.Event()
            r.event.record(s)
        r.phase = 1

    def _finish(self, r):
        res = {name: h[:k].numpy().copy() for name, (h, k) in r.host_out.items()}
        res["bases"] = res["bases"].view(np.uint32)
        res["len"] = res["len"].view(np.uint64)
        res["base_off"] = res["base_off"].view(np.uint64)
        res["cflags"] = res["cflags"].view(np.uint32)
        res["status"] = self.ctxs[r.slot].status(r.stream)
        if self.keep_outputs:
            res["full"] = cg.to_host(r.out, r.req.graph.n)
        r.req.result = res

    # -- the loop ---------------------------------------------------------

    def run(self, requests, idle_sleep=20e-6):
        """Serve `requests` (arrival times in seconds from the start) and
        return them with t_admit / t_done set; also returns the run's
        wall-clock span and peak admitted footprint."""
        import torch
        reqs = sorted(requests, key=lambda q: q.arrival)
        by_id = {q.rid: q for q in reqs}
        adm = Admission(self.slots, self.budget)
        pending = collections.deque(reqs)
        running = {}
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        while pending or adm.queue or running:
            now = time.perf_counter() - t0
            progressed = False
            while pending and pending[0].arrival <= now:
                q = pending.popleft()
                adm.push(q.rid, q.footprint)
                progressed = True
            for slot in list(running):
                r = running[slot]
                if not r.event.query():
                    continue
                progressed = True
                if r.phase == 0:
                    self._download(r)
                    continue
                self._finish(r)
                r.req.t_done = time.perf_counter() - t0
                adm.release(slot, r.req.footprint)
                del running[slot]
            for rid, slot, _ in adm.admit():
                q = by_id[rid]
                q.t_admit = time.perf_counter() - t0
                running[slot] = self._launch(q, slot)
                progressed = True
            if not progressed:
                if pending and not adm.queue and not running:
                    # idle until the next arrival
                    time.sleep(max(0.0, min(pending[0].arrival - now, 1e-3)))
                else:
                    time.sleep(idle_sleep)
        span = time.perf_counter() - t0
        return reqs, span, adm.peak


def busy_fraction(reqs, span):
    """Fraction of the run during which at least one request was admitted."""
    iv = sorted((q.t_admit, q.t_done) for q in reqs)
    tot, cur_s, cur_e = 0.0, None, None
    for s, e in iv:
        if cur_e is None or s > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = s, e
        else:
            cur_e = max(cur_e, e)
    if cur_e is not None:
        tot += cur_e - cur_s
    return tot / span if span > 0 else 0.0


def poisson_arrivals(n, rate, seed):
    """n arrival times of a Poisson process of the given rate (per second)."""
    r = np.random.default_rng(seed)
    return np.cumsum(r.exponential(1.0 / rate, size=n))

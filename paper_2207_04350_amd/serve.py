"""Serving form: continuous batching of contig-generation requests.

Requests (one string graph each) arrive over time.  A request is admitted in
arrival order when its HBM footprint fits in the budget next to the requests
already admitted; the head of the queue is never overtaken, and a request that
could never fit (or names a graph the server does not hold) is rejected on its
own while the others go on.  An admitted request's graph is uploaded from
pinned host memory and checked (cg_validate) on an intake stream, unless it is
one of the graphs made resident once (`Server.make_resident`), which stay in
HBM for the life of the server and were checked when they were made resident;
an invalid graph is rejected on its own.

Checked requests wait for a lane.  A lane is a stream with its own context and
a batch (cg_batch) whose device memory is planned anew for every wave: when a
lane is free, every checked request not yet started (up to the lane's memory)
becomes one wave, planned into the lane's batch (cg_batch_plan) and run as one
launch sequence of the batched form for all of its graphs (cg_batch_run).
Requests that arrive while a wave runs form the next wave, on the other lane,
so waves overlap on the device.  A wave that fails on the device fails its own
requests only.  When a wave is done its contigs come back to pinned host
memory: first the device-side counts of every request, then exactly the
records and bases they name.

Latency runs from arrival to the result in host memory.  Device busy time is
measured on the GPU: timing events recorded on each lane's stream around each
wave's launches, merged over the lanes.

The loop itself (`Server.run`) is plain host logic over a backend: `Device`
does the work with libcg's kernels; the tests also drive it with a CPU
stand-in to check admission, waves and failure isolation without a GPU.
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
    """HBM a request holds while it is admitted: its outputs, carved from one
    buffer (cg_job_outputs, cap_words = seq_words), and its graph unless the
    graph is resident (charged once when it was made resident).  The lanes'
    batch memory is the server's own, charged once."""
    sw = int(g.seq.shape[0])
    out = cg.job_outputs_bytes(g.n, P, sw)
    if resident:
        return out
    return out + cg.sizes(g.n, g.m, sw, P, getattr(g, "pre", None) is not None)["graph"]


# ---------------------------------------------------------------------------
# Admission core (host logic only)
# ---------------------------------------------------------------------------

class Admission:
    """FIFO admission by HBM budget.

    A request is admitted when it is at the head of the queue and the
    footprints of the admitted requests plus its own fit the budget.  The head
    is never overtaken, so a large request cannot starve; a request larger
    than the whole budget is refused at push (it could never be admitted)."""

    def __init__(self, budget):
        self.budget = int(budget)
        self.used = 0
        self.peak = 0
        self.queue = collections.deque()

    def push(self, req_id, footprint):
        """Queue a request; False (and not queued) when it can never fit."""
        if footprint > self.budget:
            return False
        self.queue.append((req_id, int(footprint)))
        return True

    def admit(self):
        """Admitted (request id, footprint) pairs, in arrival order."""
        out = []
        while self.queue and self.used + self.queue[0][1] <= self.budget:
            rid, fp = self.queue.popleft()
            self.used += fp
            self.peak = max(self.peak, self.used)
            out.append((rid, fp))
        return out

    def release(self, footprint):
        self.used -= footprint


def take_wave(ready, fits):
    """The next wave from the `ready` deque (in order): as many requests as
    `fits(list)` accepts, at least one."""
    wave = [ready.popleft()]
    while ready and fits(wave + [ready[0]]):
        wave.append(ready.popleft())
    return wave


def busy_fraction(intervals, span, kinds=None):
    """Fraction of `span` covered by the union of (start, end[, kind])
    intervals (only those of the given kinds, if any are named)."""
    iv = sorted((i[0], i[1]) for i in intervals
                if kinds is None or (len(i) > 2 and i[2] in kinds))
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


# ---------------------------------------------------------------------------
# Requests
# ---------------------------------------------------------------------------

class HostGraph:
    """A string graph in pinned host memory, as requests bring it."""

    def __init__(self, g, pin=True):
        import torch
        pinf = (lambda t: t.pin_memory()) if pin else (lambda t: t)
        conv = lambda a: pinf(torch.from_numpy(np.ascontiguousarray(a)))
        u = lambda a, dt, sdt: a.astype(dt).view(sdt)
        self.graph = g
        self.n, self.m, self.seq_words = g.n, g.m, int(g.seq.shape[0])
        self.t = dict(
            row_ptr=conv(g.row_ptr.astype(np.int32)),
            col=conv(g.col.astype(np.int32) if g.m else np.zeros(1, np.int32)),
            ovl=conv(u(g.ovl, np.uint32, np.int32) if g.m else np.zeros(1, np.int32)),
            strand=conv(g.strand.astype(np.uint8) if g.m else np.zeros(1, np.uint8)),
            read_len=conv(u(g.read_len, np.uint32, np.int32) if g.n else np.zeros(1, np.int32)),
            read_off=conv(u(g.read_off, np.uint64, np.int64) if g.n else np.zeros(1, np.int64)),
            seq=conv(u(g.seq, np.uint32, np.int32)))
        if getattr(g, "pre", None) is not None:
            z = lambda a: u(a, np.uint32, np.int32) if g.m else np.zeros(1, np.int32)
            self.t["pre"], self.t["post"] = conv(z(g.pre)), conv(z(g.post))


class Request:
    """One contig-generation request: a graph in pinned host memory (uploaded
    on admission), or one the server holds resident (`resident=True`), its
    parameters and its arrival time (seconds from the start of the run).
    After the run: `result` (the contigs, host arrays) or `error` (why the
    request was rejected or failed)."""

    def __init__(self, rid, host, P, min_reads=2, arrival=0.0, resident=False):
        self.rid, self.host, self.P, self.min_reads = rid, host, int(P), int(min_reads)
        self.graph = host.graph
        self.arrival = float(arrival)
        self.resident = bool(resident)
        self.footprint = request_footprint(self.graph, self.P, self.resident)
        self.t_admit = self.t_ready = self.t_start = self.t_done = None
        self.result = None
        self.error = None
        self.wave = None


# ---------------------------------------------------------------------------
# The loop
# ---------------------------------------------------------------------------

class Server:
    """Continuous batching of requests over a backend's lanes within `budget`
    bytes of HBM (default: the device's memory minus `reserve` and what the
    backend holds for itself)."""

    def __init__(self, backend, budget=None, reserve=16 << 30):
        self.backend = backend
        if budget is None:
            budget = backend.device_bytes() - reserve - backend.own_bytes()
        self.budget = int(budget)

    def make_resident(self, host):
        """Upload (and check) host once; requests with resident=True on it then
        run on this copy.  Its bytes leave the budget for good."""
        fp = self.backend.make_resident(host, self.budget)
        self.budget -= fp

    def close(self):
        self.backend.close()

    def run(self, requests, idle_sleep=20e-6):
        """Serve `requests` (arrival times in seconds from the start).  Returns
        them with t_admit / t_ready / t_start / t_done set and `result` or
        `error`; also the run's span (s), the peak admitted footprint and the
        device busy intervals (s from the start, merged by busy_fraction)."""
        be = self.backend
        reqs = sorted(requests, key=lambda q: q.arrival)
        by_id = {q.rid: q for q in reqs}
        adm = self.admission = Admission(self.budget)
        pending = collections.deque(reqs)
        intake = collections.deque()   # admitted, being uploaded and checked
        ready = collections.deque()    # checked, waiting for a lane
        running = {}                   # lane -> wave
        finishing = []                 # waves whose downloads are in flight
        done = n_waves = 0

        def retire(q, error=None):
            nonlocal done
            if error is not None:
                q.error = error
            q.t_done = be.now()
            if q.t_admit is not None:
                adm.release(q.footprint)
            done += 1

        be.start_clock()
        while done < len(reqs):
            now = be.now()
            progressed = False
            while pending and pending[0].arrival <= now:
                q = pending.popleft()
                progressed = True
                try:
                    why = be.refuse(q)
                except Exception as e:  # bad parameters: this request only
                    why = "refused: %s" % e
                if why is None and not adm.push(q.rid, q.footprint):
                    why = "needs %d bytes, above the %d-byte budget" % (q.footprint, adm.budget)
                if why is not None:
                    retire(q, why)
            for rid, _ in adm.admit():
                q = by_id[rid]
                q.t_admit = be.now()
                progressed = True
                try:
                    be.intake(q)
                    intake.append(q)
                except Exception as e:  # upload refused: this request only
                    retire(q, "intake: %s" % e)
            while intake and be.intake_done(intake[0]):
                q = intake.popleft()
                progressed = True
                why = be.intake_error(q)
                if why is not None:
                    retire(q, why)
                else:
                    q.t_ready = be.now()
                    ready.append(q)
            for lane in be.free_lanes(running):
                if not ready:
                    break
                wave = take_wave(ready, lambda w, lane=lane: be.fits(lane, w))
                progressed = True
                t = be.now()
                for q in wave:
                    q.t_start, q.wave = t, n_waves
                n_waves += 1
                try:
                    running[lane] = be.start_wave(lane, wave)
                except Exception as e:  # the wave failed to start: its requests only
                    for q in wave:
                        retire(q, "wave: %s" % e)
            for lane in list(running):
                w = running[lane]
                if not be.wave_done(w):
                    continue
                progressed = True
                del running[lane]
                try:
                    be.start_download(w)
                    finishing.append(w)
                except Exception as e:
                    for q in w.reqs:
                        retire(q, "wave: %s" % e)
            for w in list(finishing):
                if not be.download_done(w):
                    continue
                progressed = True
                finishing.remove(w)
                results = be.finish(w)
                for q in w.reqs:
                    r = results.get(q.rid)
                    if isinstance(r, Exception):
                        retire(q, "wave: %s" % r)
                    else:
                        q.result = r
                        retire(q)
            if not progressed:
                if pending and not (adm.queue or intake or ready or running or finishing):
                    be.sleep(max(0.0, min(pending[0].arrival - now, 1e-3)))
                else:
                    be.sleep(idle_sleep)
        span = be.now()
        return reqs, span, adm.peak, be.busy_intervals()


# ---------------------------------------------------------------------------
# The device backend
# ---------------------------------------------------------------------------

class _Wave:
    def __init__(self, lane, reqs):
        self.lane, self.reqs = lane, reqs
        self.events = None


class Device:
    """libcg on one GPU: `lanes` streams, each with its own context and a batch
    of `lane_bytes` of device memory re-planned for every wave (at most
    `max_wave` requests), and an intake stream that uploads and checks
    graphs."""

    def __init__(self, lanes=2, lane_bytes=2 << 30, max_wave=64, device="cuda",
                 vertex_tile=0, copy_block=0, persist_blocks=0):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.dev_index = self.device.index or 0
        self.n_lanes = int(lanes)
        self.lane_bytes = int(lane_bytes)
        self.max_wave = int(max_wave)
        self.vertex_tile = int(vertex_tile)
        self.ctxs = [cg.Context(self.dev_index, 0) for _ in range(self.n_lanes)]
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(self.n_lanes)]
        self.batches = [cg.Batch.empty(c, self.lane_bytes, vertex_tile, copy_block, persist_blocks)
                        for c in self.ctxs]
        self.intake_ctx = cg.Context(self.dev_index, 0)
        self.intake_stream = torch.cuda.Stream(device=self.device)
        self.resident = {}   # id(HostGraph) -> DeviceGraph
        self.graphs = {}     # rid -> DeviceGraph of an admitted request
        self.checks = {}     # rid -> (event, pinned d_bad)
        self.intervals = []
        self.t0 = None
        self.ref = None

    # -- sizes ----------------------------------------------------------------
    def device_bytes(self):
        return self.torch.cuda.get_device_properties(self.device).total_memory

    def own_bytes(self):
        return self.n_lanes * self.lane_bytes

    def refuse(self, q):
        """Why a request can never run here (None if it can)."""
        if q.resident and id(q.host) not in self.resident:
            return "names a graph that is not resident"
        # the request's share of a lane's batch memory: the figure of a batch
        # of it alone, an upper bound of its share in any wave (each table of
        # a plan is rounded up once per batch, not once per job)
        q.batch_bytes = cg.batch_bytes([(q.graph.n, q.graph.m, q.P)], self.vertex_tile)
        if q.batch_bytes > self.lane_bytes:
            return "needs %d bytes of batch memory, a lane has %d" % (q.batch_bytes,
                                                                     self.lane_bytes)
        return None

    def fits(self, lane, wave):
        return len(wave) <= self.max_wave and \
            sum(q.batch_bytes for q in wave) <= self.lane_bytes

    # -- clock and busy time ----------------------------------------------------
    def start_clock(self):
        torch = self.torch
        torch.cuda.synchronize(self.device)
        self.intervals = []
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(self.streams[0])
        self.t0 = time.perf_counter()

    def now(self):
        return time.perf_counter() - self.t0

    def sleep(self, s):
        time.sleep(s)

    def busy_intervals(self):
        """(start, end, kind) of the device's work, in seconds from the
        start, measured by events on the device: kind "kernels" for a wave's
        batched path and its result packing, "copy" for the download of its
        packed results, "intake" for a graph's upload and check."""
        return list(self.intervals)

    # -- graphs ----------------------------------------------------------------
    def _upload(self, host, stream):
        torch = self.torch
        g = host.graph
        with torch.cuda.stream(stream):
            d = {k: v.to(self.device, non_blocking=True) for k, v in host.t.items()}
        return cg.DeviceGraph.from_tensors(g.n, g.m, d, int(g.seq.shape[0]), self.device)

    def _check_async(self, dg, stream):
        torch = self.torch
        with torch.cuda.stream(stream):
            bad = torch.empty(2, dtype=torch.int64, device=self.device)
            cg.validate(self.intake_ctx, dg, bad, stream)
            h = torch.empty(2, dtype=torch.int64, pin_memory=True)
            h.copy_(bad, non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
        return ev, h

    def make_resident(self, host, budget):
        g = host.graph
        fp = graph_bytes(g.n, g.m, g.seq.shape[0], getattr(g, "pre", None) is not None)
        if id(host) in self.resident:
            return 0
        if fp > budget:
            raise ValueError("graph needs %d bytes, above the %d-byte budget left" % (fp, budget))
        dg = self._upload(host, self.intake_stream)
        ev, h = self._check_async(dg, self.intake_stream)
        ev.synchronize()
        if int(h[0]) != -1:
            raise ValueError("graph is invalid (entry %d, reason %d)" % (int(h[0]), int(h[1])))
        self.resident[id(host)] = dg
        return fp

    def intake(self, q):
        if q.resident:
            self.graphs[q.rid] = self.resident[id(q.host)]
            return
        torch = self.torch
        ev_a = torch.cuda.Event(enable_timing=True)
        ev_a.record(self.intake_stream)
        dg = self._upload(q.host, self.intake_stream)
        self.graphs[q.rid] = dg
        ev, h = self._check_async(dg, self.intake_stream)
        self.checks[q.rid] = (ev, h, ev_a)

    def intake_done(self, q):
        c = self.checks.get(q.rid)
        return c is None or c[0].query()

    def intake_error(self, q):
        c = self.checks.pop(q.rid, None)
        if c is None:
            return None
        self.intervals.append((self.ref.elapsed_time(c[2]) * 1e-3,
                               self.ref.elapsed_time(c[0]) * 1e-3, "intake"))
        bad = (int(c[1][0]), int(c[1][1]))
        if bad[0] != -1:
            self.graphs.pop(q.rid, None)
            return "invalid graph (entry %d, reason %d)" % bad
        return None

    # -- waves -----------------------------------------------------------------
    def free_lanes(self, running):
        return [k for k in range(self.n_lanes) if k not in running]

    def start_wave(self, lane, reqs):
        """Plan the wave into the lane's batch and enqueue: the batched path
        for all its requests, then their counts (cg_batch_counts) and the
        first download, of the counts alone."""
        torch = self.torch
        s = self.streams[lane]
        w = _Wave(lane, reqs)
        sizes = [cg.job_outputs_bytes(q.graph.n, q.P, int(q.graph.seq.shape[0])) for q in reqs]
        jobs = []
        with torch.cuda.stream(s):
            w.buf = torch.empty(max(sum(sizes), 256), dtype=torch.uint8, device=self.device)
            at = 0
            for q, nb in zip(reqs, sizes):
                o = cg.CarvedOutputs(w.buf, at, q.graph.n, q.P, int(q.graph.seq.shape[0]))
                at += nb
                jobs.append((self.graphs[q.rid], o, q.P, q.min_reads))
            b = self.batches[lane]
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            b.plan(jobs, s)
            ev0.record(s)
            b.run(s)
            w.d_counts = torch.empty(4 * len(reqs) + 1, dtype=torch.int64, device=self.device)
            b.counts(w.d_counts, s)
            ev1.record(s)
            w.counts = torch.empty(w.d_counts.shape, dtype=torch.int64, pin_memory=True)
            w.counts.copy_(w.d_counts, non_blocking=True)
            done = torch.cuda.Event()
            done.record(s)
        w.jobs = jobs
        w.events = (ev0, ev1, done)
        return w

    def wave_done(self, w):
        return w.events[2].query()

    def start_download(self, w):
        """The second download: every request's results, trimmed to its
        counts and packed by the library (cg_batch_pack) into one buffer."""
        torch = self.torch
        ev0, ev1, _ = w.events
        self.intervals.append((self.ref.elapsed_time(ev0) * 1e-3,
                               self.ref.elapsed_time(ev1) * 1e-3, "kernels"))
        s = self.streams[w.lane]
        w.status = self.ctxs[w.lane].status(s)
        total = int(w.counts[-1])
        with torch.cuda.stream(s):
            dst = torch.empty(max(total, 16), dtype=torch.uint8, device=self.device)
            ev2 = torch.cuda.Event(enable_timing=True)
            ev3 = torch.cuda.Event(enable_timing=True)
            ev2.record(s)
            self.batches[w.lane].pack(w.d_counts, dst, s)
            ev3.record(s)
            # the wave's own pinned buffer (torch's pinned-memory cache): the
            # requests' results are views of it, no copy on the host
            w.packed = torch.empty(max(total, 16), dtype=torch.uint8, pin_memory=True)
            w.packed.copy_(dst, non_blocking=True)
            ev4 = torch.cuda.Event(enable_timing=True)
            ev4.record(s)
            w.ev_down = torch.cuda.Event()
            w.ev_down.record(s)
        w.dst = dst
        w.pack_events = (ev2, ev3, ev4)

    def download_done(self, w):
        if not w.ev_down.query():
            return False
        ev2, ev3, ev4 = w.pack_events
        self.intervals.append((self.ref.elapsed_time(ev2) * 1e-3,
                               self.ref.elapsed_time(ev3) * 1e-3, "kernels"))
        self.intervals.append((self.ref.elapsed_time(ev3) * 1e-3,
                               self.ref.elapsed_time(ev4) * 1e-3, "copy"))
        return True

    def finish(self, w):
        packed = w.packed.numpy()
        rows = w.counts.numpy()[:-1].reshape(-1, 4)
        out = {}
        for q, row in zip(w.reqs, rows):
            res = cg.unpack_results(packed, row)
            res["status"] = w.status
            out[q.rid] = res
            self.graphs.pop(q.rid, None)
        w.buf = w.dst = w.d_counts = w.jobs = None
        return out

    def close(self):
        for b in self.batches:
            b.close()
        for c in self.ctxs:
            c.close()
        self.intake_ctx.close()
        self.batches, self.ctxs = [], []
        self.resident = {}

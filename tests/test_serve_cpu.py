"""Host logic of the serving loop: admission, footprint accounting, waves,
busy time and failure isolation (the loop driven by a CPU stand-in for the
device, on a virtual clock)."""
import numpy as np
import pytest

import synth
from paper_2207_04350_amd import serve


def test_fifo_admission_respects_budget():
    a = serve.Admission(budget=100)
    for rid, fp in (("a", 60), ("b", 30), ("c", 20), ("d", 10)):
        assert a.push(rid, fp)
    got = a.admit()
    assert [g[0] for g in got] == ["a", "b"]          # c does not fit next to a and b
    assert a.used == 90 and a.peak == 90
    a.release(60)
    assert [g[0] for g in a.admit()] == ["c", "d"]
    a.release(30)
    a.release(20)
    a.release(10)
    assert a.used == 0 and a.peak <= a.budget


def test_head_of_line_is_never_overtaken():
    a = serve.Admission(budget=100)
    a.push("x", 50)
    (_, fp_x), = a.admit()
    a.push("big", 60)          # does not fit next to x
    a.push("small", 5)         # would fit, but must wait behind big
    assert a.admit() == []
    a.release(fp_x)
    assert [g[0] for g in a.admit()] == ["big", "small"]


def test_oversized_request_is_refused_not_raised():
    a = serve.Admission(budget=10)
    assert a.push("huge", 11) is False
    assert not a.queue
    assert a.push("ok", 10) is True
    assert [g[0] for g in a.admit()] == ["ok"]


def test_take_wave():
    import collections
    ready = collections.deque(range(10))
    w = serve.take_wave(ready, lambda w: sum(w) <= 6)
    assert w == [0, 1, 2, 3] and list(ready) == [4, 5, 6, 7, 8, 9]
    # at least one, even when it alone does not fit
    w = serve.take_wave(ready, lambda w: False)
    assert w == [4]


def test_footprint_matches_the_allocations():
    """The library's footprint (cg_footprint) equals the bytes the binding
    allocates for a graph and its outputs, with and without coordinates."""
    import torch
    from paper_2207_04350_amd import cg
    g = synth.config_graph(1)
    for coords in (False, True):
        h = synth.with_alignment_ends(g) if coords else g
        for P in (8, 1000):
            dg = cg.DeviceGraph(h, "cpu")
            out = cg.Outputs(h.n, P, int(h.seq.shape[0]), "cpu")
            gb = sum(t.numel() * t.element_size() for t in (dg.row_ptr, dg.col, dg.ovl, dg.strand,
                                                             dg.read_len, dg.read_off, dg.seq,
                                                             dg.pre, dg.post) if t is not None)
            ob = sum(t.numel() * t.element_size() for t in vars(out).values()
                     if isinstance(t, torch.Tensor))
            s = cg.sizes(h.n, h.m, h.seq.shape[0], P, coords)
            assert s["graph"] == gb and s["outputs"] == ob, (coords, P)
            assert s["scratch"] == cg.footprint(h.n, h.m, P)
            assert serve.graph_bytes(h.n, h.m, h.seq.shape[0], coords) == gb
            assert serve.output_bytes(h.n, P, int(h.seq.shape[0])) == ob
            # the serving loop carves a request's outputs from one buffer,
            # every buffer at a 256-byte boundary (33 buffers)
            carved = cg.job_outputs_bytes(h.n, P, int(h.seq.shape[0]))
            assert ob <= carved <= ob + 33 * 256 and carved % 256 == 0
            assert serve.request_footprint(h, P) == gb + carved
            # a request on a resident graph holds its outputs only
            assert serve.request_footprint(h, P, resident=True) == carved


def test_batch_bytes_from_sizes():
    """cg_batch_bytes sizes a batch from (n, m, P) alone, and a wave's figure
    is at most the sum of its requests' own: the serving loop's bound."""
    from paper_2207_04350_amd import cg
    shapes = [(0, 0, 1), (1, 0, 8), (5000, 11000, 64), (200000, 60000, 64), (20000, 18433, 3)]
    one = [cg.batch_bytes([s]) for s in shapes]
    assert all(b > 0 for b in one)
    assert cg.batch_bytes(shapes) <= sum(one)
    assert cg.batch_bytes(shapes[:2]) < cg.batch_bytes(shapes)
    # larger tiles: fewer tile entries, never more bytes
    assert cg.batch_bytes(shapes, vertex_tile=1024) <= cg.batch_bytes(shapes)
    for bad in ([(-1, 0, 8)], [(10, 10, 0)], [(10, 10, 65537)], [(10, 10, 8, 7)]):
        with pytest.raises(cg.CgError):
            cg.batch_bytes(bad)
    with pytest.raises(cg.CgError):
        cg.batch_bytes([(10, 10, 8)], vertex_tile=300)


def test_busy_fraction_and_arrivals():
    assert serve.busy_fraction([(0, 1), (0.5, 2), (3, 4)], 5.0) == pytest.approx(3.0 / 5.0)
    assert serve.busy_fraction([], 5.0) == 0.0
    iv = [(0, 1, "kernels"), (0.5, 2, "copy"), (3, 3.5, "kernels")]
    assert serve.busy_fraction(iv, 4.0) == pytest.approx(2.5 / 4.0)
    assert serve.busy_fraction(iv, 4.0, ("kernels",)) == pytest.approx(1.5 / 4.0)
    a = serve.poisson_arrivals(2000, 100.0, seed=3)
    assert np.all(np.diff(a) > 0)
    assert np.array_equal(a, serve.poisson_arrivals(2000, 100.0, seed=3))
    assert abs(a[-1] / 2000 - 0.01) < 0.002      # mean gap 1/rate


# ---------------------------------------------------------------------------
# The loop on a CPU stand-in for the device
# ---------------------------------------------------------------------------

class _Host:
    """A request's graph as the loop sees it (sizes only), with switches
    that make one step fail."""

    def __init__(self, g, invalid=False, intake_raises=False, wave_raises=False,
                 result_error=False):
        self.graph = g
        self.n, self.m, self.seq_words = g.n, g.m, int(g.seq.shape[0])
        self.invalid, self.intake_raises = invalid, intake_raises
        self.wave_raises, self.result_error = wave_raises, result_error


class _FakeWave:
    def __init__(self, lane, reqs, end):
        self.lane, self.reqs, self.end = lane, reqs, end


class FakeDevice:
    """Lanes that take `wave_time(wave)` virtual seconds per wave; intake
    takes `intake_time`.  The result of a request is its id."""

    def __init__(self, lanes=2, max_wave=4, lane_bytes=1 << 40, intake_time=1e-3,
                 per_request=2e-3):
        self.lanes, self.max_wave, self.lane_bytes = lanes, max_wave, lane_bytes
        self.intake_time, self.per_request = intake_time, per_request
        self.t = 0.0
        self.intake_end = {}
        self.intervals = []
        self.waves = []
        self.resident = set()

    def device_bytes(self):
        return 1 << 40

    def own_bytes(self):
        return 0

    def make_resident(self, host, budget):
        self.resident.add(id(host))
        return 0

    def start_clock(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, s):
        self.t += max(s, 1e-5)

    def busy_intervals(self):
        return list(self.intervals)

    def refuse(self, q):
        if q.resident and id(q.host) not in self.resident:
            return "not resident"
        return None

    def fits(self, lane, wave):
        return len(wave) <= self.max_wave

    def intake(self, q):
        if q.host.intake_raises:
            raise RuntimeError("upload refused")
        self.intake_end[q.rid] = self.t + self.intake_time

    def intake_done(self, q):
        return self.t >= self.intake_end[q.rid]

    def intake_error(self, q):
        return "invalid graph" if q.host.invalid else None

    def free_lanes(self, running):
        return [k for k in range(self.lanes) if k not in running]

    def start_wave(self, lane, reqs):
        if any(q.host.wave_raises for q in reqs):
            raise RuntimeError("plan refused")
        start = self.t
        w = _FakeWave(lane, reqs, start + self.per_request * len(reqs))
        self.intervals.append((start, w.end))
        self.waves.append([q.rid for q in reqs])
        return w

    def wave_done(self, w):
        return self.t >= w.end

    def start_download(self, w):
        w.down = self.t + 1e-4

    def download_done(self, w):
        return self.t >= w.down

    def finish(self, w):
        return {q.rid: (RuntimeError("bad record") if q.host.result_error else q.rid)
                for q in w.reqs}

    def close(self):
        pass


def _small_graph():
    return synth.simulate(G=50_000, cov=10, mean_len=2000, sd_len=500, err=0.0,
                          extra_rate=0.01, seed=11)


def _run(hosts, arrivals, budget=None, **kw):
    dev = FakeDevice(**kw)
    srv = serve.Server(dev, budget=budget if budget is not None else 1 << 40)
    reqs = [serve.Request(i, h, 8, 2, float(t)) for i, (h, t) in enumerate(zip(hosts, arrivals))]
    out, span, peak = srv.run(reqs)[:3]
    return dev, srv, sorted(out, key=lambda q: q.rid), span, peak


def test_loop_batches_waves_and_finishes_everything():
    g = _small_graph()
    hosts = [_Host(g) for _ in range(10)]
    dev, srv, reqs, span, peak = _run(hosts, [0.0] * 10, max_wave=4)
    assert all(q.error is None and q.result == q.rid for q in reqs)
    # everything arrived together: waves of up to four, in arrival order
    assert [len(w) for w in dev.waves] == [4, 4, 2]
    assert sum(dev.waves, []) == list(range(10))
    assert all(q.t_done >= q.t_start >= q.t_ready >= q.t_admit >= q.arrival for q in reqs)
    assert peak <= srv.budget
    # two lanes: the first two waves overlap
    (s0, e0), (s1, e1) = dev.intervals[:2]
    assert s1 < e0
    assert 0 < serve.busy_fraction(dev.intervals, span) <= 1


def test_rejected_requests_leave_the_others_running():
    g = _small_graph()
    fp = serve.request_footprint(g, 8)
    hosts = [_Host(g) for _ in range(12)]
    hosts[1] = _Host(g, invalid=True)          # fails its check on intake
    hosts[4] = _Host(g, intake_raises=True)    # its upload is refused
    hosts[7] = _Host(g, wave_raises=True)      # its wave cannot be planned
    hosts[10] = _Host(g, result_error=True)    # its result is bad
    arrivals = [0.01 * i for i in range(12)]
    dev, srv, reqs, span, peak = _run(hosts, arrivals, budget=3 * fp, max_wave=2)
    failed = {q.rid for q in reqs if q.error is not None}
    # a wave that fails takes its own requests with it, nothing else
    wave7 = next(w for w in dev.waves + [[7]] if 7 in w)
    assert {1, 4, 7, 10} <= failed <= {1, 4, 10} | set(wave7)
    for q in reqs:
        if q.rid not in failed:
            assert q.result == q.rid
        else:
            assert q.result is None and isinstance(q.error, str)
        assert q.t_done is not None
    assert "invalid" in reqs[1].error and "intake" in reqs[4].error
    assert "wave" in reqs[7].error and "wave" in reqs[10].error
    assert peak <= srv.budget
    # every footprint was released
    assert srv.admission.used == 0 and not srv.admission.queue


def test_over_budget_request_is_rejected_alone():
    g = _small_graph()
    fp = serve.request_footprint(g, 8)
    big = synth.config_graph(1)
    assert serve.request_footprint(big, 8) > 2 * fp
    hosts = [_Host(g), _Host(big), _Host(g), _Host(g)]
    dev, srv, reqs, span, peak = _run(hosts, [0.0, 0.0, 0.001, 0.002], budget=2 * fp)
    assert reqs[1].error is not None and "budget" in reqs[1].error
    assert reqs[1].t_admit is None
    assert all(reqs[k].result == k for k in (0, 2, 3))
    assert peak <= 2 * fp


def test_resident_request_on_unknown_graph_is_rejected_alone():
    g = _small_graph()
    dev = FakeDevice()
    srv = serve.Server(dev, budget=1 << 40)
    known = _Host(g)
    srv.make_resident(known)
    reqs = [serve.Request(0, known, 8, 2, 0.0, resident=True),
            serve.Request(1, _Host(g), 8, 2, 0.0, resident=True),
            serve.Request(2, known, 8, 2, 0.0, resident=True)]
    out = sorted(srv.run(reqs)[0], key=lambda q: q.rid)
    assert out[0].result == 0 and out[2].result == 2
    assert out[1].result is None and "resident" in out[1].error


def test_head_waits_for_budget_and_later_requests_queue_behind_it():
    g = _small_graph()
    fp = serve.request_footprint(g, 8)
    big = synth.config_graph(1)
    fpb = serve.request_footprint(big, 8)
    hosts = [_Host(g), _Host(big), _Host(g)]
    dev, srv, reqs, span, peak = _run(hosts, [0.0, 0.0005, 0.0006], budget=fpb + fp // 2,
                                      per_request=5e-3)
    # the big one waits for the first to leave, the last waits behind it
    assert reqs[1].t_admit >= reqs[0].t_done
    assert reqs[2].t_admit >= reqs[1].t_admit
    assert all(q.result == q.rid for q in reqs)
    assert peak <= srv.budget

"""Host logic of the serving loop: admission, footprint accounting, busy time."""
import numpy as np
import pytest

import synth
from paper_2207_04350_amd import serve


def test_fifo_admission_respects_slots_and_budget():
    a = serve.Admission(slots=2, budget=100)
    for rid, fp in (("a", 60), ("b", 30), ("c", 20), ("d", 10)):
        a.push(rid, fp)
    got = a.admit()
    assert [g[0] for g in got] == ["a", "b"]          # two slots
    assert a.used == 90 and a.peak == 90
    a.release(got[0][1], 60)
    got2 = a.admit()
    assert [g[0] for g in got2] == ["c"]              # one slot free
    a.release(got[1][1], 30)
    a.release(got2[0][1], 20)
    assert [g[0] for g in a.admit()] == ["d"]
    assert a.used == 10 and a.peak <= a.budget


def test_head_of_line_is_never_overtaken():
    a = serve.Admission(slots=4, budget=100)
    a.push("big", 90)
    a.push("small", 5)
    assert [g[0] for g in a.admit()] == ["big", "small"]
    a = serve.Admission(slots=4, budget=100)
    a.push("x", 50)
    (_, slot_x, fp_x), = a.admit()
    a.push("big", 60)          # does not fit next to x
    a.push("small", 5)         # would fit, but must wait behind big
    assert a.admit() == []
    a.release(slot_x, fp_x)
    assert [g[0] for g in a.admit()] == ["big", "small"]
    assert sorted(a.free) == [2, 3]


def test_oversized_request_is_rejected():
    a = serve.Admission(slots=1, budget=10)
    with pytest.raises(ValueError):
        a.push("huge", 11)


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
            assert serve.request_footprint(h, P) == gb + ob
            # a request on a resident graph holds its outputs only
            assert serve.request_footprint(h, P, resident=True) == ob


def test_busy_fraction_and_arrivals():
    class R:
        def __init__(self, a, d):
            self.t_admit, self.t_done = a, d
    reqs = [R(0, 1), R(0.5, 2), R(3, 4)]
    assert serve.busy_fraction(reqs, 5.0) == pytest.approx(3.0 / 5.0)
    a = serve.poisson_arrivals(2000, 100.0, seed=3)
    assert np.all(np.diff(a) > 0)
    assert np.array_equal(a, serve.poisson_arrivals(2000, 100.0, seed=3))
    assert abs(a[-1] / 2000 - 0.01) < 0.002      # mean gap 1/rate

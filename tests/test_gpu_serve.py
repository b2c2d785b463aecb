"""GPU: the serving loop batches each wave of admitted requests into one
cg_batch plan.  Every request's result is the same alone and in a concurrent
mix and equals the oracle (a request above 50 Mbp among them), admission
never exceeds its HBM budget, and an invalid graph is rejected on its own."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pool():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_04350_amd import cg, serve
    cg.lib()
    ps = synth.request_params(40)
    small = [p for p in ps if p["G"] <= 12_000_000][:6]
    big = [p for p in ps if p["G"] >= 50_000_000][:1]
    assert big, "the request mix needs a graph of at least 50 Mbp"
    graphs = [synth.simulate(**p) for p in small + big]
    graphs.append(synth.config_graph(1))
    return [serve.HostGraph(g) for g in graphs]


def _P(h):
    return 64 if h.n > 5000 else 8


def _requests(serve, pool, arrivals, order, resident=False):
    return [serve.Request(i, pool[k], _P(pool[k]), 2, float(t), resident=resident)
            for i, (k, t) in enumerate(zip(order, arrivals))]


def _server(serve, budget=None, **kw):
    kw.setdefault("lane_bytes", 1 << 30)
    return serve.Server(serve.Device(**kw), budget=budget)


def _same(a, b):
    keys = [k for k in a if k not in ("full",)]
    return all(np.array_equal(a[k], b[k]) for k in keys if not np.isscalar(a[k])) and \
        a["status"] == b["status"] == 0


def _check_oracle(pool, reqs):
    for k in range(len(pool)):
        q = next(q for q in reqs if q.host is pool[k])
        want = oracle.run(pool[k].graph, P=q.P, min_reads=2)["contigs"]
        got = q.result
        assert got is not None, (k, q.error)
        assert np.array_equal(got["bases"], want["bases"]), k
        for name in ("label", "bin", "start", "n_reads", "len", "base_off", "layout_vid",
                     "layout_rev"):
            assert np.array_equal(got[name].astype(np.int64), want[name].astype(np.int64)), (k, name)


def test_alone_and_mix_identical_and_match_oracle(pool):
    from paper_2207_04350_amd import serve
    rng = np.random.default_rng(9)
    order = list(range(len(pool))) + list(rng.integers(0, len(pool), 14))
    # alone: one lane, waves of one request
    _say("alone", len(order))
    srv = _server(serve, lanes=1, max_wave=1)
    alone, _, _, _ = srv.run(_requests(serve, pool, [0.0] * len(order), order))
    srv.close()
    assert all(q.error is None for q in alone), [q.error for q in alone if q.error]
    # mix: two lanes, waves of up to 64, arrivals in a tight Poisson burst
    _say("mix")
    srv = _server(serve, lanes=2, max_wave=64)
    mix, span, peak, busy = srv.run(_requests(serve, pool,
                                              serve.poisson_arrivals(len(order), 2000.0, 4), order))
    srv.close()
    assert all(q.error is None for q in mix), [q.error for q in mix if q.error]
    assert 0 < serve.busy_fraction(busy, span) <= 1
    # the burst is served in waves of several requests
    sizes = np.bincount([q.wave for q in mix])
    assert sizes.max() > 1 and len(sizes) < len(mix)
    for qa, qm in zip(sorted(alone, key=lambda q: q.rid), sorted(mix, key=lambda q: q.rid)):
        assert _same(qa.result, qm.result), qa.rid
    _say("oracle")
    _check_oracle(pool, alone)


def test_budget_is_never_exceeded(pool):
    from paper_2207_04350_amd import serve
    order = [len(pool) - 1] * 3 + list(range(len(pool)))
    fps = [serve.request_footprint(pool[k].graph, _P(pool[k])) for k in order]
    budget = max(fps) + min(fps)          # room for the largest and one small at most
    srv = _server(serve, budget=budget, lanes=2, max_wave=64)
    reqs, span, peak, _ = srv.run(_requests(serve, pool, [0.0] * len(order), order))
    srv.close()
    assert peak <= budget
    assert all(q.result is not None and q.result["status"] == 0 for q in reqs)
    assert all(q.t_done >= q.t_start >= q.t_ready >= q.t_admit >= q.arrival for q in reqs)


def test_resident_graphs_alone_and_mix(pool):
    """Graphs made resident once: requests on them (outputs only) give the
    same bytes alone and in a mix as requests that upload their graph, and
    the budget charged for the resident copies comes off the total."""
    from paper_2207_04350_amd import serve
    rng = np.random.default_rng(10)
    order = list(range(len(pool))) + list(rng.integers(0, len(pool), 10))
    srv = _server(serve, lanes=1, max_wave=1)
    up, _, _, _ = srv.run(_requests(serve, pool, [0.0] * len(order), order))
    srv.close()
    _say("resident mix", len(order))
    srv = _server(serve, lanes=2, max_wave=64)
    before = srv.budget
    for h in pool:
        srv.make_resident(h)
    assert srv.budget == before - sum(serve.graph_bytes(h.n, h.m, h.seq_words) for h in pool)
    mix, span, peak, _ = srv.run(_requests(serve, pool,
                                           serve.poisson_arrivals(len(order), 2000.0, 5), order,
                                           resident=True))
    srv.close()
    assert peak <= srv.budget
    for qa, qm in zip(sorted(up, key=lambda q: q.rid), sorted(mix, key=lambda q: q.rid)):
        assert qa.error is None and qm.error is None, (qa.error, qm.error)
        assert _same(qa.result, qm.result), qa.rid


def test_invalid_graph_is_rejected_alone(pool):
    """A graph that fails cg_validate (an entry names a read out of range)
    is rejected on intake; the requests around it complete unchanged."""
    from paper_2207_04350_amd import serve
    import copy
    g = copy.copy(pool[0].graph)
    g.col = g.col.copy()
    g.col[0] = g.n + 7
    bad = serve.HostGraph(g)
    hosts = [pool[0], bad, pool[1], pool[0]]
    reqs = [serve.Request(i, h, _P(h), 2, 0.0) for i, h in enumerate(hosts)]
    srv = _server(serve, lanes=2, max_wave=64)
    out, _, _, _ = srv.run(reqs)
    srv.close()
    out = sorted(out, key=lambda q: q.rid)
    assert out[1].result is None and "invalid" in out[1].error
    srv = _server(serve, lanes=1, max_wave=1)
    ref, _, _, _ = srv.run([serve.Request(i, h, _P(h), 2, 0.0)
                            for i, h in enumerate([pool[0], pool[1]])])
    srv.close()
    ref = sorted(ref, key=lambda q: q.rid)
    assert _same(out[0].result, ref[0].result) and _same(out[3].result, ref[0].result)
    assert _same(out[2].result, ref[1].result)

"""GPU: every request's result is the same alone and in a concurrent mix,
equals the oracle, and admission never exceeds its HBM budget."""
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
    ps = [p for p in synth.request_params(40) if p["G"] <= 12_000_000][:6]
    graphs = [synth.simulate(**p) for p in ps]
    graphs.append(synth.config_graph(1))
    return [serve.HostGraph(g) for g in graphs]


def _requests(serve, pool, arrivals, order):
    return [serve.Request(i, pool[k], 64 if pool[k].n > 5000 else 8, 2, float(t))
            for i, (k, t) in enumerate(zip(order, arrivals))]


def _server(serve, pool, **kw):
    return serve.Server(max(h.n for h in pool), max(h.m for h in pool), 64, **kw)


def _same(a, b):
    keys = [k for k in a if k not in ("full",)]
    return all(np.array_equal(a[k], b[k]) for k in keys if not np.isscalar(a[k])) and \
        a["status"] == b["status"] == 0


def test_alone_and_mix_identical_and_match_oracle(pool):
    from paper_2207_04350_amd import serve
    rng = np.random.default_rng(9)
    order = list(range(len(pool))) + list(rng.integers(0, len(pool), 14))
    # alone: one slot, every request runs by itself
    _say("alone", len(order))
    srv = _server(serve, pool, slots=1)
    alone, _, _ = srv.run(_requests(serve, pool, [0.0] * len(order), order))
    srv.close()
    # mix: four slots, arrivals in a tight Poisson burst
    _say("mix")
    srv = _server(serve, pool, slots=4)
    mix, span, peak = srv.run(_requests(serve, pool, serve.poisson_arrivals(len(order), 2000.0, 4),
                                        order))
    srv.close()
    assert serve.busy_fraction(mix, span) > 0
    for qa, qm in zip(sorted(alone, key=lambda q: q.rid), sorted(mix, key=lambda q: q.rid)):
        assert _same(qa.result, qm.result), qa.rid
    # and each distinct graph against the oracle
    for k in range(len(pool)):
        q = next(q for q in alone if q.host is pool[k])
        want = oracle.run(pool[k].graph, P=q.P, min_reads=2)["contigs"]
        got = q.result
        assert np.array_equal(got["bases"], want["bases"]), k
        for name in ("label", "bin", "start", "n_reads", "len", "base_off", "layout_vid",
                     "layout_rev"):
            assert np.array_equal(got[name].astype(np.int64), want[name].astype(np.int64)), (k, name)


def test_budget_is_never_exceeded(pool):
    from paper_2207_04350_amd import serve
    order = [len(pool) - 1] * 3 + list(range(len(pool)))
    fps = [serve.request_footprint(pool[k].graph, 64 if pool[k].n > 5000 else 8) for k in order]
    budget = max(fps) + min(fps)          # room for the largest and one small at most
    srv = _server(serve, pool, slots=4, budget=budget)
    reqs, span, peak = srv.run(_requests(serve, pool, [0.0] * len(order), order))
    srv.close()
    assert peak <= budget
    assert all(q.result is not None and q.result["status"] == 0 for q in reqs)
    assert all(q.t_done >= q.t_admit >= q.arrival for q in reqs)


def test_resident_graphs_alone_and_mix(pool):
    """Graphs made resident once: requests on them (outputs only) give the
    same bytes alone and in a mix as requests that upload their graph, and
    the budget charged for the resident copies comes off the total."""
    from paper_2207_04350_amd import serve
    rng = np.random.default_rng(10)
    order = list(range(len(pool))) + list(rng.integers(0, len(pool), 10))

    def reqs(arrivals, resident):
        return [serve.Request(i, pool[k], 64 if pool[k].n > 5000 else 8, 2, float(t),
                              resident=resident)
                for i, (k, t) in enumerate(zip(order, arrivals))]

    srv = _server(serve, pool, slots=1)
    up, _, _ = srv.run(reqs([0.0] * len(order), False))
    srv.close()
    _say("resident mix", len(order))
    srv = _server(serve, pool, slots=4)
    before = srv.budget
    for h in pool:
        srv.make_resident(h)
    assert srv.budget == before - sum(serve.graph_bytes(h.n, h.m, h.seq_words) for h in pool)
    mix, span, peak = srv.run(reqs(serve.poisson_arrivals(len(order), 2000.0, 5), True))
    srv.close()
    assert peak <= srv.budget
    for qa, qm in zip(sorted(up, key=lambda q: q.rid), sorted(mix, key=lambda q: q.rid)):
        assert _same(qa.result, qm.result), qa.rid

"""Bases-weighted LPT: a component weighs the total length of its reads.

GreedyPartitioning is unchanged (Section 4.3: decreasing weights, least
loaded bin); only the weights differ from the paper's read counts.  The bin
boundaries of the induced numbering keep counting reads."""
import math

import numpy as np
import pytest

import oracle
import synth
from tests import brute


def _masking_graph(golden, lens):
    ex = golden["masking"]
    reads = [np.zeros(L, np.uint8) for L in lens]
    return synth.graph_from_edges(reads, [(a, b, 50, 0, 0) for a, b in ex["edges"]])


def test_weights_can_reorder_the_partition(golden):
    """Hand-worked: the components of the masking example, {0,1}, {3,4,5} and
    {6,7}, with reads of 1000, 100 and 500 bases weigh 2000, 300 and 1000.
    By bases (P = 2): 2000 -> bin 0, 1000 -> bin 1, 300 -> bin 1 (loads 2000,
    1300); by reads (sizes 2, 3, 2): 3 -> bin 0, 2 -> bin 1, 2 -> bin 1."""
    lens = [1000, 1000, 200, 100, 100, 100, 500, 500]
    g = _masking_graph(golden, lens)
    rb = oracle.run(g, P=2, weight="bases")["parts"]
    got = {int(l): int(b) for l, b in zip(rb["comp_label"], rb["comp_bin"])}
    assert got == {0: 0, 6: 1, 3: 1}
    assert rb["bin_load"].tolist() == [2000, 1300]
    rr = oracle.run(g, P=2, weight="reads")["parts"]
    assert {int(l): int(b) for l, b in zip(rr["comp_label"], rr["comp_bin"])} == {3: 0, 0: 1, 6: 1}
    assert rr["bin_load"].tolist() == [3, 4]


def test_weights_are_the_components_read_lengths():
    g = synth.config_graph(1)
    r = oracle.run(g, P=8, weight="bases")
    label, parts = r["label"], r["parts"]
    for k, c in enumerate(parts["comp_label"]):
        members = np.nonzero(label == c)[0]
        assert len(members) == parts["comp_size"][k]
    w = oracle.component_weights(g, label, parts["label_comp"], parts["comp_size"], "bases")
    for k, c in enumerate(parts["comp_label"]):
        assert int(w[k]) == int(g.read_len[label == c].sum())
    loads = np.zeros(8, np.uint64)
    np.add.at(loads, parts["comp_bin"], w)
    assert np.array_equal(loads, parts["bin_load"])


def test_weighted_lpt_against_exhaustive_optimum():
    rng = np.random.default_rng(5)
    for _ in range(150):
        P = int(rng.integers(1, 5))
        nc = int(rng.integers(0, 8))
        w = rng.integers(1, 5000, size=nc).astype(np.uint64)
        labels = np.sort(rng.choice(1000, size=nc, replace=False)).astype(np.int32)
        comp_bin, loads = oracle.lpt(w, labels, P)
        opt = brute.lpt_opt([int(x) for x in w], P)
        mk = int(loads.max()) if P else 0
        assert mk * 3 * P <= (4 * P - 1) * opt
        assert mk >= max(int(w.max(initial=0)), math.ceil(int(w.sum()) / P))


def test_equal_read_lengths_give_the_read_count_partition():
    rng = np.random.default_rng(9)
    for _ in range(40):
        g = synth.adversarial(rng)
        h = synth.StringGraph(**{k: getattr(g, k) for k in ("n", "m", "row_ptr", "col", "ovl",
                                                           "strand", "read_len", "read_off",
                                                           "seq")})
        if g.n == 0 or int(g.read_len.min()) < 2:
            continue
        h.read_len = np.full(g.n, int(g.read_len.min()), np.uint32)
        h.ovl = np.minimum(g.ovl, int(h.read_len[0]) - 1).astype(np.uint32)
        if oracle.validate(h)[0] != -1:
            continue
        a = oracle.run(h, P=3, min_reads=1, weight="reads")["parts"]
        b = oracle.run(h, P=3, min_reads=1, weight="bases")["parts"]
        assert np.array_equal(a["comp_bin"], b["comp_bin"])


def test_bin_boundaries_count_reads_under_any_weight():
    g = synth.config_graph(1)
    for weight in ("reads", "bases"):
        r = oracle.run(g, P=8, weight=weight)
        parts, local = r["parts"], r["local"]
        per_bin = np.zeros(8, np.int64)
        np.add.at(per_bin, parts["comp_bin"], parts["comp_size"])
        assert np.array_equal(np.diff(local["bin_vptr"]), per_bin)


def test_bases_weights_beyond_range_are_rejected():
    g = synth.config_graph(1)
    r = oracle.run(g, P=8)
    big = synth.StringGraph(**{k: getattr(g, k) for k in ("n", "m", "row_ptr", "col", "ovl",
                                                         "strand", "read_len", "read_off", "seq")})
    big.read_len = g.read_len.copy()
    k = int(np.argmax(r["parts"]["comp_size"]))
    members = np.nonzero(r["label"] == r["parts"]["comp_label"][k])[0]
    big.read_len[members[:2]] = np.uint32(3_000_000_000)
    with pytest.raises(ValueError):
        oracle.component_weights(big, r["label"], r["parts"]["label_comp"], r["parts"]["comp_size"],
                                 "bases")

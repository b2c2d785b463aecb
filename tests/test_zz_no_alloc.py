"""The allocation-free entry point (cg_contig_generation_noalloc) gives the
same outputs as the five context calls, on two calls in a row (the second on
a smaller graph), and refuses a graph beyond its static scratch."""
import ctypes
import sys

import numpy as np
import pytest

import synth
from tests.parity import mismatches

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _with_ctx(cg, g, P, mr, weight):
    ctx = cg.Context.for_graph(g.n, g.m, P)
    dg = cg.DeviceGraph(g, "cuda")
    out = cg.Outputs(g.n, P, g.seq_words, "cuda")
    cg.run_path(ctx, dg, out, P, mr, weight=weight)
    got = cg.to_host(out, g.n)
    assert ctx.status() == 0
    ctx.close()
    return got


def test_noalloc_matches_the_context_calls():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2207_04350_amd import cg
    cg.lib()
    cases = [(synth.config_graph(2), 64, 2, "reads"),
             (synth.config_graph(1), 8, 2, "bases"),
             (synth.with_alignment_ends(synth.config_graph(1), np.random.default_rng(3), 3), 3, 1,
              "reads")]
    status = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    for g, P, mr, w in cases:
        _say("noalloc case n=%d m=%d P=%d min_reads=%d weight=%s" % (g.n, g.m, P, mr, w))
        want = _with_ctx(cg, g, P, mr, w)
        dg = cg.DeviceGraph(g, "cuda")
        out = cg.Outputs(g.n, P, g.seq_words, "cuda")
        for t in (out.flags, out.label, out.perm, out.bases, out.c_len):
            t.fill_(-1 if t.dtype != torch.uint8 else 255)
        cg.contig_generation_noalloc(dg, out, P, mr, weight=w, d_status=status)
        got = cg.to_host(out, g.n)
        assert mismatches(got, want) == []
        assert int(status.item()) == 0


def test_noalloc_refuses_a_graph_beyond_its_scratch():
    from paper_2207_04350_amd import cg
    n = 1 << 20
    assert cg.footprint(n, 2 * n, 64) > cg.NOALLOC_SCRATCH_BYTES
    g = cg.CgGraph()
    g.n, g.m = n, 2 * n
    buf = (ctypes.c_int32 * 8)()
    p = ctypes.cast(buf, ctypes.c_void_p)      # checked on the host only, never read
    g.row_ptr = g.col = g.ovl = g.strand = g.read_len = g.read_off = g.seq = p
    parts = cg.CgParts(*([p] * 9))
    local = cg.CgLocal(*([p] * 6))
    contigs = cg.CgContigs(*([p] * 11), 8, p)
    rc = cg.lib().cg_contig_generation_noalloc(ctypes.byref(g), 64, 2, 0, p, p, p,
                                               ctypes.byref(parts), ctypes.byref(local),
                                               ctypes.byref(contigs), None, None)
    assert rc == cg.CG_EUNSUPPORTED
    assert b"allocation-free" in cg.lib().cg_last_error()

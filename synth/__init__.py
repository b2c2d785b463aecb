"""Seeded synthetic inputs (genomes, reads, string graphs) for tests and benchmarks."""
from .gen import (CONFIGS, SEED_BASE, StringGraph, adversarial, batch_graphs, batch_params,
                  with_alignment_ends, overlap_graph,
                  build_helper, config_graph, csr_from_edges, decode, encode, graph_from_edges,
                  pack_reads, request_params, simulate, unpack_read)

__all__ = ["CONFIGS", "SEED_BASE", "StringGraph", "adversarial", "batch_graphs", "batch_params",
           "with_alignment_ends", "overlap_graph",
           "build_helper", "config_graph", "csr_from_edges", "decode", "encode",
           "graph_from_edges", "pack_reads", "request_params", "simulate", "unpack_read"]

"""Seeded synthetic graph generators shared by the tests, the bench and the oracle runs.

This module only produces inputs: an undirected simple graph in CSR form plus one
non-overlapping community label per vertex.  It holds none of the scoring
arithmetic of the robust-spanner method; both the HIP path and the CPU oracle
receive the same arrays from here.
"""
from .graphs import (  # noqa: F401
    Graph,
    canonical_csr,
    sbm,
    lfr,
    random_small,
    from_edges,
    cfg_sbm_small,
    cfg_lfr_1m,
    cfg_lfr_20m,
    cfg_batch_graph,
    cfg_batch,
    pack_batch,
    graph_stats,
    cached,
)

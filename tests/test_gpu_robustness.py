"""Reachable communities on the GPU (absolute AWCC, Section VII-B) equal the
oracle's breadth-first searches, on the loaded graph and after rounds of
edge and vertex removal (the disruption model of the experiments)."""
import sys

import numpy as np
import pytest

import oracle
from rsgen import from_edges, lfr, sbm

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[reach]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("make", [lambda: lfr(8000, 6.0, 200, 0.2, seed=51, cmin=10, cmax=600),
                                  lambda: sbm([300] * 10, 0.004, 0.0004, seed=52)],
                         ids=["lfr_8k_sparse", "sbm_fragmented"])
def test_reach_matches_bfs_under_removals(make):
    import paper_2508_01485_amd as rs
    g = make()
    rng = np.random.default_rng(5)
    u, v = g.edges()
    alive_e = np.ones(u.size, bool)
    alive_v = np.ones(g.n, bool)
    src = rng.choice(g.n, 24, replace=False)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h)
        for step in range(6):
            if step:
                if step % 2:
                    live = np.flatnonzero(alive_e)
                    pick = rng.choice(live, live.size // 10, replace=False)
                    alive_e[pick] = False
                    rs.rs_apply_removals(h, edges=np.stack([u[pick], v[pick]], 1))
                else:
                    live = np.flatnonzero(alive_v)
                    pick = rng.choice(live, live.size // 20, replace=False)
                    alive_v[pick] = False
                    alive_e &= alive_v[u] & alive_v[v]
                    rs.rs_apply_removals(h, vertices=pick)
            got = rs.rs_reachable_communities(h, src)
            cur = from_edges(g.n, np.stack([u[alive_e], v[alive_e]], 1), g.labels)
            exp = oracle.reachable_communities(cur, src, alive=alive_v)
            assert np.array_equal(got, exp), (step, np.flatnonzero(got != exp)[:5])
            # the one-hop reading is the row length ell of each source
            ell = rs.rs_read_vertex_counts(h)["ell"][src]
            hop = [len(set(cur.labels[cur.col[cur.off[x]:cur.off[x + 1]]].tolist())) for x in src]
            assert np.array_equal(ell, hop), step
            _say(f"step {step}: {int(alive_e.sum())} edges, mean reach {got.mean():.2f}")
    finally:
        h.free()


def test_reach_errors_and_empty():
    import paper_2508_01485_amd as rs
    g = sbm([50, 50], 0.1, 0.01, seed=53)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        assert rs.rs_reachable_communities(h, []).size == 0
        with pytest.raises(rs.RSError, match="out of range"):
            rs.rs_reachable_communities(h, [g.n])
        with pytest.raises(rs.RSError, match="n_sources"):
            rs.rs_reachable_communities(h, np.zeros(1025, np.int32))
    finally:
        h.free()

"""rs_reachable_communities_static, the form of rs_reachable_communities that
allocates nothing (for callers that cannot allocate device memory: stream
capture, serving loops): its counts equal the allocating entry point's, on
two calls in a row that share the device's static scratch, the second on a
smaller graph with fewer sources (so stale scratch contents would show)."""
import numpy as np
import pytest

from rsgen import lfr, sbm

pytestmark = pytest.mark.gpu


def _check(rs, g, n_src, seed):
    rng = np.random.default_rng(seed)
    u, v = g.edges()
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h)
        # break the graph into pieces first, so components differ per source
        pick = rng.choice(u.size, u.size // 3, replace=False)
        rs.rs_apply_removals(h, edges=np.stack([u[pick], v[pick]], 1))
        src = rng.choice(g.n, n_src, replace=False).astype(np.int32)
        a = rs.rs_reachable_communities(h, src)
        b = rs.rs_reachable_communities_static(h, src)
        assert np.array_equal(a, b), np.flatnonzero(a != b)[:10]
        assert a.max() > 0
        return a
    finally:
        h.free()


def test_static_reach_equals_allocating_form():
    import paper_2508_01485_amd as rs
    big = lfr(20000, 8.0, 300, 0.25, seed=61, cmin=10, cmax=800)
    small = sbm([150] * 8, 0.02, 0.002, seed=62)
    assert small.n < big.n
    _check(rs, big, 600, 1)
    _check(rs, small, 37, 2)


def test_static_reach_refuses_oversized_and_bad_args():
    import paper_2508_01485_amd as rs
    g = sbm([40, 40], 0.1, 0.02, seed=63)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        assert rs.rs_reachable_communities_static(h, []).size == 0
        with pytest.raises(rs.RSError, match="out of range"):
            rs.rs_reachable_communities_static(h, [g.n])
        with pytest.raises(rs.RSError, match="n_sources"):
            rs.rs_reachable_communities_static(h, np.zeros(1025, np.int32))
    finally:
        h.free()


def test_static_reach_refuses_a_graph_beyond_its_scratch():
    """9,000,000 vertices need 36 MB of component labels: more than the
    32 MiB array, so the call is refused before anything runs."""
    import paper_2508_01485_amd as rs
    from rsgen import from_edges
    n = 9_000_000
    g = from_edges(n, [(0, 1), (1, 2)], np.zeros(n, np.int32))
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        with pytest.raises(rs.RSError) as ei:
            rs.rs_reachable_communities_static(h, [0])
        assert ei.value.status == 3 and "static scratch" in ei.value.detail
        assert rs.rs_reachable_communities(h, [0, 5]).tolist() == [1, 0]
    finally:
        h.free()

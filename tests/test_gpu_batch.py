"""The batched form: several graphs loaded as one disjoint union and scored in
one pass (each with its own w_max, Algorithm 1 Step 2 per graph) give, vertex
for vertex, the bits of each graph loaded alone: per-vertex integers, the own
weight, the triad counts, R and the raw score, and a per-graph top-k equal to
each lone graph's rs_topk; and every graph of a batch matches the CPU oracle
run on that graph alone."""
import sys

import numpy as np
import pytest

from rsgen import lfr, random_small, sbm

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[batch]", *a, flush=True)
    sys.stdout.flush()


def _graphs():
    """Uneven sizes and kinds, including an edgeless graph, a one-vertex
    graph, an empty graph and arbitrary label values."""
    gs = [
        lfr(6000, 12.0, 200, 0.25, seed=70, cmin=10, cmax=300),
        random_small(40, 0.2, 4, seed=71, label_values=[9, 400, 17, 3]),
        sbm([300, 200, 150, 90], 0.08, 0.01, seed=72),
        random_small(25, 0.0, 3, seed=73),           # no edges
        lfr(3000, 10.0, 150, 0.4, seed=74, cmin=8, cmax=200),
        random_small(1, 0.0, 1, seed=75),            # one vertex
        random_small(0, 0.0, 1, seed=76),            # no vertices
        sbm([64] * 12, 0.3, 0.02, seed=77),
        lfr(9000, 14.0, 400, 0.3, seed=78, cmin=10, cmax=500),
        random_small(120, 0.1, 9, seed=79),
    ]
    return gs


def _union(gs):
    vo = np.concatenate([[0], np.cumsum([g.n for g in gs])]).astype(np.int64)
    eo = np.concatenate([[0], np.cumsum([g.nnz for g in gs])]).astype(np.int64)
    off = np.concatenate([[0]] + [g.off[1:] + eo[i] for i, g in enumerate(gs)]).astype(np.int64)
    col = np.concatenate([g.col.astype(np.int64) + vo[i] for i, g in enumerate(gs)]).astype(np.int32)
    lab = np.concatenate([g.labels for g in gs]).astype(np.int32)
    return vo, off, col, lab


def _alone(rs, g, k):
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h)
        ids, sc = rs.rs_topk(h, k)
        out = {"ids": ids, "scores": sc, "R": rs.rs_read_scores(h), "raw": rs.rs_read_scores(h, raw=True)}
        out.update(rs.rs_read_vertex_counts(h))
    finally:
        h.free()
    return out


@pytest.mark.parametrize("k", [1, 7, 32])
def test_batch_equals_alone(k):
    import paper_2508_01485_amd as rs
    gs = _graphs()
    vo, off, col, lab = _union(gs)
    _say(f"k={k}: {len(gs)} graphs, n={vo[-1]}, nnz={off[-1]}")
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        rs.rs_score(h)
        ids, sc, cnt = rs.rs_topk_batch(h, k)
        R = rs.rs_read_scores(h)
        raw = rs.rs_read_scores(h, raw=True)
        vc = rs.rs_read_vertex_counts(h)
    finally:
        h.free()
    for i, g in enumerate(gs):
        a, b = vo[i], vo[i + 1]
        ref = _alone(rs, g, k) if g.n > 0 else None
        if ref is None:
            assert cnt[i] == 0
            continue
        assert R[a:b].tobytes() == ref["R"].tobytes(), i
        assert raw[a:b].tobytes() == ref["raw"].tobytes(), i
        for key in ("border", "ell", "dprime", "tI", "tII"):
            assert np.array_equal(vc[key][a:b], ref[key]), (i, key)
        assert vc["w_own"][a:b].tobytes() == ref["w_own"].tobytes(), i
        c = int(cnt[i])
        assert c == ref["ids"].size, (i, c, ref["ids"].size)
        assert np.array_equal(ids[i, :c], ref["ids"]), i
        assert sc[i, :c].tobytes() == ref["scores"].tobytes(), i
    _say(f"k={k}: every graph's bits equal its lone load")


def test_batch_of_many_tiny_graphs():
    """Hundreds of graphs of 0-60 vertices (many per row tile), k above most
    graph sizes: counts = live vertices, lists equal the lone loads."""
    import paper_2508_01485_amd as rs
    rng = np.random.default_rng(81)
    gs = [random_small(int(rng.integers(0, 61)), float(rng.uniform(0.05, 0.5)), int(rng.integers(1, 7)), seed=900 + i)
          for i in range(300)]
    vo, off, col, lab = _union(gs)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        rs.rs_score(h)
        ids, sc, cnt = rs.rs_topk_batch(h, 32)
        R = rs.rs_read_scores(h)
    finally:
        h.free()
    for i, g in enumerate(gs):
        assert cnt[i] == min(32, g.n), i
        if g.n == 0:
            continue
        ref = _alone(rs, g, 32)
        assert R[vo[i]:vo[i + 1]].tobytes() == ref["R"].tobytes(), i
        assert np.array_equal(ids[i, :cnt[i]], ref["ids"]), i
        assert sc[i, :cnt[i]].tobytes() == ref["scores"].tobytes(), i
    _say("300 tiny graphs: identical to their lone loads")


def test_batch_with_a_graph_above_the_segment_limit():
    """A graph of more than 64 top-k segments (65,536 vertices) sends the
    batch to the one-wavefront-per-graph top-k; results still equal the lone
    loads.  Segment-boundary sizes (1,024, 2,048 and 1,025 vertices) ride along."""
    import paper_2508_01485_amd as rs
    gs = [lfr(70000, 8.0, 150, 0.3, seed=82, cmin=20, cmax=2000),
          random_small(1024, 0.01, 5, 83), random_small(2048, 0.005, 7, 84), random_small(1025, 0.01, 3, 85)]
    for big in (True, False):
        sel = gs if big else gs[1:]
        vo, off, col, lab = _union(sel)
        h = rs.rs_load_batch(vo, off, col, lab)
        try:
            rs.rs_score(h)
            ids, sc, cnt = rs.rs_topk_batch(h, 25)
        finally:
            h.free()
        for i, g in enumerate(sel):
            ref = _alone(rs, g, 25)
            c = int(cnt[i])
            assert c == ref["ids"].size, (big, i)
            assert np.array_equal(ids[i, :c], ref["ids"]), (big, i)
            assert sc[i, :c].tobytes() == ref["scores"].tobytes(), (big, i)
    _say("batches with and without a graph above the segment limit: identical to lone loads")


def test_batch_rescore_is_stable():
    """A second score pass on a batch gives the same bits (replayed graphs)."""
    import paper_2508_01485_amd as rs
    gs = _graphs()
    vo, off, col, lab = _union(gs)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        rs.rs_score(h)
        r1 = rs.rs_read_scores(h).copy()
        t1 = rs.rs_topk_batch(h, 16)
        rs.rs_score(h)
        r2 = rs.rs_read_scores(h)
        t2 = rs.rs_topk_batch(h, 16)
    finally:
        h.free()
    assert r1.tobytes() == r2.tobytes()
    for x, y in zip(t1, t2):
        assert x.tobytes() == y.tobytes()


def test_reachable_communities_on_a_batch():
    """Components never span graphs, so each source's count on the batch
    equals the oracle's search inside its own graph."""
    import oracle
    import paper_2508_01485_amd as rs
    gs = [random_small(60, 0.03, 5, 91), sbm([40, 30, 30], 0.05, 0.01, seed=92), random_small(1, 0.0, 1, 93),
          lfr(2000, 5.0, 60, 0.3, seed=94, cmin=10, cmax=200)]
    vo, off, col, lab = _union(gs)
    rng = np.random.default_rng(95)
    src = rng.choice(int(vo[-1]), 40, replace=False)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        got = rs.rs_reachable_communities(h, src)
        with pytest.raises(rs.RSError, match="not applied to a batch"):
            rs.rs_restrict_to_targets(h, 2)
    finally:
        h.free()
    for s_, c in zip(src, got):
        gi = int(np.searchsorted(vo, s_, side="right") - 1)
        exp = oracle.reachable_communities(gs[gi], [int(s_ - vo[gi])])[0]
        assert c == exp, (s_, gi, c, exp)


def test_batch_errors():
    import paper_2508_01485_amd as rs
    gs = _graphs()[:3]
    vo, off, col, lab = _union(gs)
    # an edge that joins graph 0 and graph 1
    col2 = col.copy()
    col2[0] = vo[1]
    with pytest.raises(rs.RSError, match="joins two graphs"):
        rs.rs_load_batch(vo, off, col2, lab)
    with pytest.raises(rs.RSError, match="0..n"):
        rs.rs_load_batch(vo[:-1], off, col, lab)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        with pytest.raises(rs.RSError, match="before rs_score"):
            rs.rs_topk_batch(h, 4)
        rs.rs_score(h)
        with pytest.raises(rs.RSError, match="k must be"):
            rs.rs_topk_batch(h, 33)
        with pytest.raises(rs.RSError, match="not applied to a batch"):
            rs.rs_apply_removals(h, vertices=[0])
    finally:
        h.free()
    p = rs.rs_load_graph(gs[0].off, gs[0].col, gs[0].labels)
    try:
        rs.rs_score(p)
        p.n_graphs = 1
        with pytest.raises(rs.RSError, match="not a batch"):
            rs.rs_topk_batch(p, 4)
    finally:
        p.free()


def _check_batch_against_oracle(rs, gs, k):
    """Every graph of the batch against the oracle on that graph alone:
    integers exact, R within 1e-6 (zero exactly where the oracle's is), the
    per-graph top-k position by position outside near-tie classes."""
    import oracle
    from tests.parity import REL, rel_close, topk_matches
    vo, off, col, lab = _union(gs)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        rs.rs_score(h)
        ids, sc, cnt = rs.rs_topk_batch(h, k)
        R = rs.rs_read_scores(h)
        vc = rs.rs_read_vertex_counts(h)
    finally:
        h.free()
    exempt = 0
    for i, g in enumerate(gs):
        a, b = vo[i], vo[i + 1]
        if g.n == 0:
            assert cnt[i] == 0
            continue
        o = oracle.score(g)
        for key in ("ell", "dprime", "tI", "tII"):
            assert np.array_equal(np.asarray(vc[key][a:b], np.int64), np.asarray(o[key], np.int64)), (i, key)
        assert np.array_equal(vc["border"][a:b].astype(np.uint8), o["border"]), i
        rel_close(R[a:b], o["R"], REL)
        o_ids, o_sc = oracle.topk(o["R"], k)
        c = int(cnt[i])
        assert c == o_ids.size, (i, c, o_ids.size)
        exempt += topk_matches(ids[i, :c], o_ids, o["R"], k)
        rel_close(sc[i, :c], R[a:b][ids[i, :c]], 0.0)
    return exempt


def test_batch_matches_oracle():
    """The uneven test batch and the first 48 graphs of the 4,096-graph
    batched workload (seeds 1000 + g), each checked against the oracle."""
    import paper_2508_01485_amd as rs
    from rsgen import cfg_batch_graph
    for gs, k in ((_graphs(), 20), ([cfg_batch_graph(i) for i in range(48)], 20)):
        ex = _check_batch_against_oracle(rs, gs, k)
        _say(f"{len(gs)} graphs (n={sum(g.n for g in gs)}) equal the oracle's, {ex} near-tie positions")

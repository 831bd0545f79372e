"""GPU parity: the HIP path through the C ABI against the CPU oracle."""
import os
import sys

import numpy as np
import pytest

import oracle
from rsgen import cfg_lfr_1m, cfg_sbm_small, from_edges, lfr, random_small, sbm
from tests.parity import compare, gpu_run, rel_close

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def rs():
    import paper_2508_01485_amd as m
    return m


def _check(g, k, name, flags=0):
    _say(f"[parity] {name}: n={g.n} nnz={g.nnz} k={k} flags={flags}")
    gpu = gpu_run(g, k, flags=flags)
    ora = oracle.score(g, rows=True)
    diag = compare(g, gpu, ora, k)
    _say(f"[parity] {name}: ok {diag}")
    return gpu, ora, diag


def test_k4_closed_form(rs):
    g = from_edges(4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], [7, 1, 5, 3])
    gpu, ora, _ = _check(g, 4, "k4")
    np.testing.assert_allclose(gpu["R"], 2 / (3 * np.log2(3)), rtol=1e-12)
    assert list(gpu["ids"]) == [0, 1, 2, 3]


def test_sbm_small_config(rs):
    g = cfg_sbm_small(0)
    _check(g, 20, "sbm n=2000")


@pytest.mark.parametrize("seed", range(12))
def test_random_small_graphs(rs, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 300))
    g = random_small(n, float(rng.uniform(0.005, 0.3)), int(rng.integers(1, 12)), 40_000 + seed,
                     label_values=rng.permutation(100_000)[:12] * 7)
    _check(g, int(rng.integers(1, n + 5)), f"gnp seed={seed}")


def test_empty_and_edgeless(rs):
    g = from_edges(0, np.zeros((0, 2)), [])
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    rs.rs_score(h)
    ids, sc = rs.rs_topk(h, 5)
    assert ids.size == 0 and rs.rs_read_scores(h).size == 0
    h.free()
    g = from_edges(9, np.zeros((0, 2)), [3, 1, 4, 1, 5, 9, 2, 6, 5])
    gpu, ora, _ = _check(g, 4, "edgeless")
    assert list(gpu["ids"]) == [0, 1, 2, 3]


def test_single_and_two_communities(rs):
    for k in (1, 2):
        g = random_small(120, 0.1, k, 77 + k)
        gpu, ora, _ = _check(g, 10, f"{k} communities")
        assert np.all(gpu["R"] == 0.0)


def test_hubs_and_long_rows(rs):
    """Rows longer than a wavefront (multi-chunk path) and a hub of degree > 2048."""
    rng = np.random.default_rng(5)
    n = 6000
    base = random_small(n, 0.0008, 40, 55)
    u, v = base.edges()
    hub_edges = [(0, int(x)) for x in rng.choice(np.arange(1, n), 2500, replace=False)]
    mid_edges = [(1, int(x)) for x in rng.choice(np.arange(2, n), 300, replace=False)]
    e = np.concatenate([np.stack([u, v], 1), np.array(hub_edges), np.array(mid_edges)])
    g = from_edges(n, e, base.labels)
    _check(g, 50, "hubs")


def test_hub_runs_cross_stream_groups(rs):
    """Hub rows whose community runs are longer than one streaming group
    (2,048 entries), so runs stay open across group boundaries."""
    rng = np.random.default_rng(6)
    n = 12000
    labels = np.concatenate([np.full(3000, 1), np.full(2500, 2), np.full(2600, 3),
                             rng.integers(4, 40, n - 8100)])
    rng.shuffle(labels)
    base = random_small(n, 0.0006, 5, 66)
    u, v = base.edges()
    hubs = [(0, int(x)) for x in rng.choice(np.arange(1, n), 7000, replace=False)]
    hubs += [(1, int(x)) for x in rng.choice(np.arange(2, n), 4500, replace=False)]
    hubs += [(2, int(x)) for x in rng.choice(np.arange(3, n), 1500, replace=False)]
    g = from_edges(n, np.concatenate([np.stack([u, v], 1), np.array(hubs)]), labels)
    _check(g, 40, "hub runs")


def test_score_hub_beyond_lds_staging(rs):
    """Two adjacent hubs (hub-hub pairs) with foreign lists of ~10,000 entries
    and > 4,096 distinct neighbour communities: too large for a score unit's
    LDS list, so their chunks read u's side from HBM; keys beyond one 16-key
    read take the multi-level search."""
    rng = np.random.default_rng(8)
    n = 15000
    labels = rng.integers(0, 7000, n)
    base = random_small(n, 0.0002, 5, 88)
    u, v = base.edges()
    hubs = [(0, int(x)) for x in rng.choice(np.arange(1, n), 12000, replace=False)]
    hubs += [(1, int(x)) for x in rng.choice(np.arange(2, n), 9500, replace=False)]
    hubs += [(0, 1)]
    g = from_edges(n, np.concatenate([np.stack([u, v], 1), np.array(hubs)]), labels)
    _check(g, 60, "score hubs beyond LDS")


def test_wide_offsets_path(rs):
    """The 64-bit edge-offset kernels (used for nnz > 2^31) on small graphs:
    row hubs, score hubs beyond LDS staging, a triangle-rich LFR graph and
    removals; integer results bit-identical to the 32-bit form."""
    rng = np.random.default_rng(31)
    n = 9000
    labels = rng.integers(0, 3000, n)
    base = random_small(n, 0.0005, 5, 131)
    u, v = base.edges()
    hubs = [(0, int(x)) for x in rng.choice(np.arange(1, n), 6000, replace=False)]
    hubs += [(1, int(x)) for x in rng.choice(np.arange(2, n), 2600, replace=False)]
    hubs += [(0, 1)]
    g1 = from_edges(n, np.concatenate([np.stack([u, v], 1), np.array(hubs)]), labels)
    g2 = lfr(20000, 16.0, 600, 0.2, seed=13, cmin=20, cmax=1500)
    for name, g, k in (("hubs", g1, 40), ("lfr n=20000", g2, 100)):
        wide, _, _ = _check(g, k, f"wide offsets, {name}", flags=rs.RS_LOAD_WIDE_OFFSETS)
        narrow = gpu_run(g, k)
        for key in ("border", "ell", "dprime", "tI", "tII", "ids"):
            assert np.array_equal(wide[key], narrow[key]), key
        rel_close(wide["R"], narrow["R"], 1e-12)
    # removals on the wide form equal a fresh load of the mutated graph
    gu, gv = g2.edges()
    pick = rng.choice(gu.size, 300, replace=False)
    h = rs.rs_load_graph(g2.off, g2.col, g2.labels, flags=rs.RS_LOAD_WIDE_OFFSETS)
    rs.rs_score(h)
    rs.rs_apply_removals(h, edges=np.stack([gu[pick], gv[pick]], 1), vertices=[5, 77])
    c1 = rs.rs_read_vertex_counts(h)
    R1 = rs.rs_read_scores(h)
    h.free()
    keep = np.ones(gu.size, bool)
    keep[pick] = False
    dead = np.zeros(g2.n, bool)
    dead[[5, 77]] = True
    keep &= ~dead[gu] & ~dead[gv]
    g3 = from_edges(g2.n, np.stack([gu[keep], gv[keep]], 1), g2.labels)
    ora = oracle.score(g3)
    rel_close(R1, ora["R"], 1e-6)
    assert np.array_equal(c1["tI"], ora["tI"]) and np.array_equal(c1["tII"], ora["tII"])


def test_lfr_small(rs):
    g = lfr(30000, 20.0, 800, 0.2, seed=3, cmin=20, cmax=2000)
    _check(g, 100, "lfr n=30000")


def test_topk_sort_widths(rs):
    """Top-k sizes on both sides of the common path's bound: up to k = 10,240
    the final list and the threshold bin are ranked together by counting
    across workgroups; beyond it (10,241 and 12,000, where the top-k also
    reaches into the zero scores) the general path ranks the bin, then the
    final list."""
    g = lfr(30000, 20.0, 800, 0.2, seed=4, cmin=20, cmax=2000)
    ora = oracle.score(g)
    from tests.parity import topk_matches
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h)
        for k in (700, 1100, 2100, 3500, 6000, 10240, 10241, 12000):
            ids, sc = rs.rs_topk(h, k)
            exp_ids, _ = oracle.topk(ora["R"], k)
            used = topk_matches(ids, exp_ids, ora["R"], k)
            _say(f"[parity] top-{k}: ok, {used} near-tie positions")
            rel_close(sc, ora["R"][ids], 1e-6)
    finally:
        h.free()


def test_sbm_uneven_dense_inter(rs):
    g = sbm([5, 40, 300, 25, 80, 2], 0.3, 0.05, 9)
    _check(g, 30, "sbm uneven")


def test_many_exact_ties_small_class(rs):
    """400 disjoint K4s with the same labels: every vertex has the same score;
    the top-k must follow caller ids (tie class smaller than the pairwise cap)."""
    edges, labels = [], []
    for c in range(400):
        b = 4 * c
        edges += [(b + i, b + j) for i in range(4) for j in range(i + 1, 4)]
        labels += [0, 1, 2, 3]
    g = from_edges(1600, edges, labels)
    gpu, ora, _ = _check(g, 37, "k4 x400")
    assert list(gpu["ids"]) == list(range(37))


def test_many_exact_ties_refine_path(rs):
    """A tie class larger than the pairwise ranker (5,000 K4s = 20,000 equal
    scores) goes through the digit-by-digit refinement."""
    edges, labels = [], []
    for c in range(5000):
        b = 4 * c
        edges += [(b + i, b + j) for i in range(4) for j in range(i + 1, 4)]
        labels += [0, 1, 2, 3]
    g = from_edges(20000, edges, labels)
    gpu, ora, _ = _check(g, 123, "k4 x5000")
    assert list(gpu["ids"]) == list(range(123))


def test_k_larger_than_nonzero_scores(rs):
    """More requested than non-zero scores: zero-score vertices follow by id."""
    g = random_small(200, 0.01, 6, 123)
    gpu, ora, _ = _check(g, 200, "k=n")
    assert gpu["ids"].size == 200


def test_deterministic_bits(rs):
    g = lfr(20000, 15.0, 400, 0.3, seed=11, cmin=10, cmax=500)
    a = gpu_run(g, 50)
    b = gpu_run(g, 50)
    assert a["R"].tobytes() == b["R"].tobytes()
    assert np.array_equal(a["ids"], b["ids"])


def test_device_resident_input_and_torch_stream(rs):
    import torch
    g = cfg_sbm_small(1)
    dev = torch.device("cuda:0")
    s = torch.cuda.Stream()
    h = rs.rs_load_graph(torch.from_numpy(g.off).to(dev), torch.from_numpy(g.col).to(dev),
                         torch.from_numpy(g.labels).to(dev), stream=s)
    rs.rs_score(h)
    ids, _ = rs.rs_topk(h, 20)
    R = rs.rs_read_scores(h)
    h.free()
    ora = oracle.score(g)
    rel_close(R, ora["R"], 1e-6)
    assert list(ids) == list(oracle.topk(ora["R"], 20)[0])


def test_removals_equal_fresh_load(rs):
    """rs_apply_removals then reading == loading the mutated graph from scratch,
    and both match the oracle.  Integer results are identical; scores agree to
    1e-12 relative (the tiles and out-list orientation are fixed at load time,
    so a vertex's floating-point summation order can differ from a fresh
    load's)."""
    g = lfr(20000, 12.0, 300, 0.25, seed=21, cmin=10, cmax=400)
    rng = np.random.default_rng(4)
    u, v = g.edges()
    pick = rng.choice(u.size, 500, replace=False)
    rem_e = np.stack([u[pick], v[pick]], 1)
    rem_e = np.concatenate([rem_e, rem_e[:20, ::-1], [[0, 0], [1, 2]]])  # repeats, reversed, absent
    rem_v = rng.choice(g.n, 30, replace=False)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    rs.rs_score(h)
    res = rs.rs_apply_removals(h, edges=rem_e, vertices=rem_v)
    R1 = rs.rs_read_scores(h)
    c1 = rs.rs_read_vertex_counts(h)
    rs.rs_score(h)  # a full pass on the mutated resident graph reproduces the same bits
    assert rs.rs_read_scores(h).tobytes() == R1.tobytes()
    ids1, _ = rs.rs_topk(h, 100)
    h.free()
    # the mutated graph, built on the host
    keep = np.ones(u.size, bool)
    keep[pick] = False
    dead = np.zeros(g.n, bool)
    dead[rem_v] = True
    keep &= ~dead[u] & ~dead[v]
    g2 = from_edges(g.n, np.stack([u[keep], v[keep]], 1), g.labels)
    assert res["edges_removed"] == u.size - int(keep.sum())
    assert res["vertices_removed"] == 30
    h2 = rs.rs_load_graph(g2.off, g2.col, g2.labels)
    rs.rs_score(h2)
    R2 = rs.rs_read_scores(h2)
    c2 = rs.rs_read_vertex_counts(h2)
    h2.free()
    rel_close(R1, R2, 1e-12)
    for key in ("border", "ell", "dprime", "tI", "tII"):
        assert np.array_equal(c1[key], c2[key]), key
    ora = oracle.score(g2)
    rel_close(R1, ora["R"], 1e-6)
    alive = (~dead).astype(np.uint8)
    exp_ids, _ = oracle.topk(ora["R"], 100, alive=alive)
    from tests.parity import topk_matches
    topk_matches(ids1, exp_ids, ora["R"], 100, alive=alive)
    assert not np.isin(ids1, rem_v).any()


def test_removals_on_triangle_rich_hubs(rs):
    """Removals that delete edges between communities of a triangle-rich graph
    with hubs (so oriented out-lists lose entries), including a hub vertex,
    then re-score: equal to the oracle on the mutated graph."""
    rng = np.random.default_rng(12)
    n = 3000
    labels = rng.integers(0, 60, n)
    base = random_small(n, 0.004, 5, 91)
    u, v = base.edges()
    hubs = [(h, int(x)) for h in range(4) for x in rng.choice(np.arange(4, n), 900, replace=False)]
    hubs += [(0, 1), (0, 2), (1, 2), (2, 3)]
    g = from_edges(n, np.concatenate([np.stack([u, v], 1), np.array(hubs)]), labels)
    gu, gv = g.edges()
    cross = np.nonzero(labels[gu] != labels[gv])[0]
    pick = rng.choice(cross, 400, replace=False)
    rem_e = np.concatenate([np.stack([gu[pick], gv[pick]], 1), [[0, 1], [1, 2]]])
    rem_v = np.array([3, 17, 2999])
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    rs.rs_score(h)
    rs.rs_apply_removals(h, edges=rem_e, vertices=rem_v)
    R1 = rs.rs_read_scores(h)
    c1 = rs.rs_read_vertex_counts(h)
    ids1, _ = rs.rs_topk(h, 50)
    h.free()
    keep = np.ones(gu.size, bool)
    ekey = set(map(tuple, np.sort(rem_e, 1).tolist()))
    keep &= np.array([(a, b) not in ekey for a, b in zip(gu.tolist(), gv.tolist())])
    dead = np.zeros(n, bool)
    dead[rem_v] = True
    keep &= ~dead[gu] & ~dead[gv]
    g2 = from_edges(n, np.stack([gu[keep], gv[keep]], 1), labels)
    ora = oracle.score(g2)
    rel_close(R1, ora["R"], 1e-6)
    assert np.array_equal(c1["tI"], ora["tI"]) and np.array_equal(c1["tII"], ora["tII"])
    assert int(ora["tI"].sum()) > 0
    alive = (~dead).astype(np.uint8)
    exp_ids, _ = oracle.topk(ora["R"], 50, alive=alive)
    from tests.parity import topk_matches
    topk_matches(ids1, exp_ids, ora["R"], 50, alive=alive)


def test_removals_next_to_hubs_chain_equals_full_pass(rs):
    """Removals next to score hubs of several chunks (foreign lists beyond
    the LDS size and within it) whose own rows stay intact, so that only the
    chunks holding pairs that read a changed row rerun: the pair with the
    changed neighbour, the triangles through it, and the a_v run sums.  Four
    batches in a row on one handle (no full pass in between), each equal bit
    for bit to a second handle of the same schedule that runs a full pass
    after the same removals; the last state also against the oracle."""
    rng = np.random.default_rng(31)
    n = 8000
    labels = rng.integers(0, 60, n).astype(np.int32)
    m = 6 * n
    a = rng.integers(6, n, m)
    b = rng.integers(6, n, m)
    sizes = [3000, 2400, 1800, 1100, 700, 400]  # four hubs beyond 1024 foreign entries, two within
    hub_e = [(h, int(x)) for h, sz in enumerate(sizes) for x in rng.choice(np.arange(6, n), sz, replace=False)]
    g = from_edges(n, np.concatenate([np.stack([a, b], 1), np.array(hub_e)]), labels)
    gu, gv = g.edges()
    cross = np.flatnonzero((labels[gu] != labels[gv]) & (gu >= 6) & (gv >= 6))
    h_inc = rs.rs_load_graph(g.off, g.col, g.labels)
    h_ref = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h_inc)
        rs.rs_score(h_ref)
        keep = np.ones(gu.size, bool)
        for step in range(4):
            live = cross[keep[cross]]
            pick = rng.choice(live, 300, replace=False)
            e = np.stack([gu[pick], gv[pick]], 1)
            res = rs.rs_apply_removals(h_inc, edges=e)
            assert res["edges_removed"] == 300
            rs.rs_apply_removals(h_ref, edges=e)
            rs.rs_score(h_ref)
            keep[pick] = False
            R1, R2 = rs.rs_read_scores(h_inc), rs.rs_read_scores(h_ref)
            assert R1.tobytes() == R2.tobytes(), f"batch {step}"
            c1, c2 = rs.rs_read_vertex_counts(h_inc), rs.rs_read_vertex_counts(h_ref)
            for key in ("border", "ell", "dprime", "tI", "tII"):
                assert np.array_equal(c1[key], c2[key]), (step, key)
            _say(f"[parity] hub-neighbour batch {step}: {res['affected']} vertices affected, bits equal")
        g2 = from_edges(n, np.stack([gu[keep], gv[keep]], 1), labels)
        o2 = oracle.score(g2)
        rel_close(R1, o2["R"], 1e-6)
        assert np.array_equal(c1["tI"], o2["tI"]) and np.array_equal(c1["tII"], o2["tII"])
        assert int(o2["tI"].sum()) > 0
    finally:
        h_inc.free()
        h_ref.free()


def _apply_and_check_full(rs, h):
    """After rs_apply_removals: a full pass gives the same bits and counts."""
    R1 = rs.rs_read_scores(h)
    c1 = rs.rs_read_vertex_counts(h)
    k1 = rs.rs_read_counts(h)
    rs.rs_score(h)
    assert rs.rs_read_scores(h).tobytes() == R1.tobytes()
    c2 = rs.rs_read_vertex_counts(h)
    for key in ("border", "ell", "dprime", "tI", "tII"):
        assert np.array_equal(c1[key], c2[key]), key
    k2 = rs.rs_read_counts(h)
    for key in ("n_border", "m_inter", "sum_ell", "sum_tI", "sum_tII", "omega_max"):
        assert k1[key] == k2[key], key
    return R1, c1, k1


def test_incremental_removals(rs):
    """rs_apply_removals re-scores only the vertices that depend on the
    removed edges, and the result equals a full pass bit for bit: one edge,
    a batch that moves w_max (rescaling every score), then several batches
    in a row, each against the oracle on the mutated graph."""
    g = lfr(20000, 14.0, 400, 0.25, seed=33, cmin=10, cmax=500)
    rng = np.random.default_rng(7)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        rs.rs_score(h)
        w0 = rs.rs_read_counts(h)["omega_max"]
        gu, gv = g.edges()
        keep = np.ones(gu.size, bool)
        dead = np.zeros(g.n, bool)
        # one cross-community edge
        cross = np.flatnonzero(g.labels[gu] != g.labels[gv])
        i0 = int(cross[0])
        res = rs.rs_apply_removals(h, edges=[[gu[i0], gv[i0]]])
        assert res["edges_removed"] == 1 and 0 < res["affected"] < g.n // 10, res
        keep[i0] = False
        _apply_and_check_full(rs, h)
        # the vertices holding the largest weights lose their edges: w_max moves
        ora = oracle.score(g, rows=True)
        ho = ora["hist_off"]
        seg = np.zeros(g.n)
        nz = np.flatnonzero(ho[1:] > ho[:-1])
        seg[nz] = np.maximum.reduceat(ora["hist_w"], ho[:-1][nz])
        vmax = np.where(ora["border"] > 0, np.maximum(ora["w_own"], seg), 0.0)
        top = np.argsort(-vmax, kind="stable")[:20]
        res = rs.rs_apply_removals(h, vertices=top)
        dead[top] = True
        keep &= ~dead[gu] & ~dead[gv]
        _, _, k = _apply_and_check_full(rs, h)
        assert k["omega_max"] != w0
        # three more batches
        for b in range(3):
            live = np.flatnonzero(keep)
            pick = rng.choice(live, 150, replace=False)
            rs.rs_apply_removals(h, edges=np.stack([gu[pick], gv[pick]], 1))
            keep[pick] = False
            R1, c1, _ = _apply_and_check_full(rs, h)
            g2 = from_edges(g.n, np.stack([gu[keep], gv[keep]], 1), g.labels)
            o2 = oracle.score(g2)
            rel_close(R1, o2["R"], 1e-6)
            assert np.array_equal(c1["tI"], o2["tI"]) and np.array_equal(c1["tII"], o2["tII"])
            _say(f"[parity] incremental batch {b}: ok")
    finally:
        h.free()


def test_graph_replay_equals_eager(rs):
    """The pass and top-k replayed from captured HIP graphs give the same
    bits as eager launches (RS_GRAPHS=0), replay after replay, with eager
    work, removals and synchronisations in between; with timing on (eager
    launches with events) every launch is counted, and replays resume after."""
    g = lfr(12000, 12.0, 300, 0.25, seed=44, cmin=10, cmax=400)
    os.environ["RS_GRAPHS"] = "0"
    try:
        he = rs.rs_load_graph(g.off, g.col, g.labels)
    finally:
        del os.environ["RS_GRAPHS"]
    hg = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        gu, gv = g.edges()
        rng = np.random.default_rng(3)
        for step in range(6):
            for h in (he, hg):
                rs.rs_score(h)
            ids_e, sc_e = rs.rs_topk(he, 200)
            ids_g, sc_g = rs.rs_topk(hg, 200)
            assert np.array_equal(ids_e, ids_g) and sc_e.tobytes() == sc_g.tobytes(), step
            assert rs.rs_read_scores(he).tobytes() == rs.rs_read_scores(hg).tobytes(), step
            if step == 2:  # eager removals between replays
                pick = rng.choice(gu.size, 100, replace=False)
                for h in (he, hg):
                    rs.rs_apply_removals(h, edges=np.stack([gu[pick], gv[pick]], 1))
            if step == 4:  # another k between replays
                a, _ = rs.rs_topk(he, 37)
                b, _ = rs.rs_topk(hg, 37)
                assert np.array_equal(a, b)
        rs.rs_set_timing(hg, True)
        rs.rs_read_timings(hg)
        for _ in range(3):
            rs.rs_score(hg)
            rs.rs_topk(hg, 200)
        t = rs.rs_read_timings(hg)
        rs.rs_set_timing(hg, False)
        assert t["k_rows"][1] == 3 and t["k_score"][1] == 3 and t["k_topk_hist"][1] == 3, t
        assert t["k_rows"][0] > 0.0
        rs.rs_score(he)
        rs.rs_score(hg)
        assert np.array_equal(rs.rs_topk(he, 200)[0], rs.rs_topk(hg, 200)[0])
        assert rs.rs_read_scores(he).tobytes() == rs.rs_read_scores(hg).tobytes()
    finally:
        he.free()
        hg.free()


def test_error_paths_on_device(rs):
    g = cfg_sbm_small(2)
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    with pytest.raises(rs.RSError) as ei:
        rs.rs_topk(h, 5)
    assert ei.value.status == rs.RS_ERR_STATE
    rs.rs_score(h)
    with pytest.raises(rs.RSError) as ei:
        rs.rs_apply_removals(h, edges=[[0, g.n]])
    assert ei.value.status == rs.RS_ERR_RANGE
    before = rs.rs_read_scores(h)
    assert rs.rs_read_scores(h).tobytes() == before.tobytes()  # unchanged after the refused batch
    h.free()
    os.environ["RS_FAULT_ALLOC"] = "3"
    try:
        with pytest.raises(rs.RSError) as ei:
            rs.rs_load_graph(g.off, g.col, g.labels)
        assert ei.value.status == rs.RS_ERR_NOMEM
    finally:
        del os.environ["RS_FAULT_ALLOC"]


@pytest.mark.slow
def test_lfr_1m_full_parity(rs):
    _say("[parity] generating LFR n=1e6")
    g = cfg_lfr_1m(0)
    _check(g, 1000, "lfr n=1e6")

"""The autotuner of the pass's schedule (tile sizes and degree bins,
rs_set_tiling / rs_autotune and paper_2508_01485_amd.autotune): a re-cut
schedule gives the same results -- every integer exactly, the same top-k, R
within 1e-12 (a vertex that moves between a tile and a hub sums its terms in
another order) -- rs_autotune keeps the fastest candidate, and a degree
signature seen before is served from the cache."""
import sys

import numpy as np
import pytest

from rsgen import cfg_batch_graph, lfr, pack_batch
from tests.parity import rel_close

pytestmark = pytest.mark.gpu

SMALL = {"row_entries": 512, "row_vertices": 128, "score_pairs": 64, "score_vertices": 64, "hub_list": 256}
MID = {"row_entries": 1024, "row_vertices": 256, "score_pairs": 128, "score_vertices": 128, "hub_list": 512}


def _say(*a):
    print("[autotune]", *a, flush=True)
    sys.stdout.flush()


def _read(rs, h, k, batch):
    rs.rs_score(h)
    out = {"R": rs.rs_read_scores(h)}
    out.update(rs.rs_read_vertex_counts(h))
    if batch:
        out["ids"], out["sc"], out["cnt"] = rs.rs_topk_batch(h, k)
    else:
        out["ids"], out["sc"] = rs.rs_topk(h, k)
    return out


def _same(a, b):
    """Integers exact, R within 1e-12, and the top-k lists equal except where
    scores tie within 1e-12 (another summation order may order those
    differently): there the lists hold the same scores and, within each
    such run, the same ids."""
    for key in ("border", "ell", "dprime", "tI", "tII"):
        assert np.array_equal(a[key], b[key]), key
    rel_close(a["R"], b["R"], 1e-12)
    ia, ib = np.atleast_2d(a["ids"]), np.atleast_2d(b["ids"])
    sa, sb = np.atleast_2d(a["sc"]), np.atleast_2d(b["sc"])
    assert ia.shape == ib.shape
    rel_close(sa, sb, 1e-12)
    for r in range(ia.shape[0]):
        diff = np.flatnonzero(ia[r] != ib[r])
        for i in diff:  # a reordered near-tie: both lists hold the other id at a tied position
            near = np.flatnonzero(np.abs(sb[r] - sb[r][i]) <= 1e-12 * max(abs(sb[r][i]), 1e-300))
            assert ia[r][i] in ib[r][near] and ib[r][i] in ia[r][near], (r, i)


def test_recut_schedules_give_the_same_results():
    import paper_2508_01485_amd as rs
    gs = [cfg_batch_graph(i) for i in range(24)]
    vo, off, col, lab = pack_batch(gs)
    h = rs.rs_load_batch(vo, off, col, lab)
    try:
        from paper_2508_01485_amd import autotune
        assert rs.rs_get_tiling(h) == autotune.DEFAULT
        ref = _read(rs, h, 20, True)
        for t in (SMALL, MID, autotune.DEFAULT):
            rs.rs_set_tiling(h, t)
            assert rs.rs_get_tiling(h) == t
            with pytest.raises(rs.RSError) as ei:  # re-cut: to be scored again
                rs.rs_read_scores(h)
            assert ei.value.status == 6
            _same(_read(rs, h, 20, True), ref)
            _say(f"{t}: same results")
        with pytest.raises(rs.RSError) as ei:
            rs.rs_set_tiling(h, dict(SMALL, row_entries=4096))
        assert ei.value.status == 1
    finally:
        h.free()


def test_autotune_keeps_the_fastest_and_caches(tmp_path):
    import paper_2508_01485_amd as rs
    from paper_2508_01485_amd import autotune
    g = lfr(40000, 14.0, 2000, 0.25, seed=91, cmin=10, cmax=800)
    cache = str(tmp_path / "tiling.json")
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        ref = _read(rs, h, 100, False)
        best, ms = rs.rs_autotune(h, [SMALL, MID, autotune.DEFAULT], 2)
        assert ms.size == 3 and np.all(ms > 0) and best == int(np.argmin(ms))
        assert rs.rs_get_tiling(h) == [SMALL, MID, autotune.DEFAULT][best]
        _same(_read(rs, h, 100, False), ref)  # scored again with the kept cut-offs
        res = autotune.tune(h, g.off, cache_path=cache, reps=2)
        assert not res["cached"] and rs.rs_get_tiling(h) == res["tiling"]
        _same(_read(rs, h, 100, False), ref)
        _say("searched", res)
    finally:
        h.free()
    h = rs.rs_load_graph(g.off, g.col, g.labels)
    try:
        res2 = autotune.tune(h, g.off, cache_path=cache)
        assert res2["cached"] and res2["tiling"] == res["tiling"] and rs.rs_get_tiling(h) == res["tiling"]
        _same(_read(rs, h, 100, False), ref)
    finally:
        h.free()
